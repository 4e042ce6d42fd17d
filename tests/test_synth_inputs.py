"""The seeded input recipe (CPU): the 640x480 rooms' depth carries the stated
Kinect-like axial noise, sigma(z) = 0.0012 + 0.0019 (z - 0.4)^2 m, is
quantised to whole millimetres, and drops 2% of the pixels."""
import numpy as np

import synth


def render_pair(seed=7):
    rng = np.random.default_rng(1905020822)
    prims = np.stack(synth._furnished_room(rng))
    poses = synth._orbit_trajectory(rng, 2)
    W, H = 640, 480
    args = (np.repeat(prims[None], 2, 0), poses, W, H, 525.0, 525.0, (W - 1) / 2.0, (H - 1) / 2.0, seed)
    exact, _, _ = synth.render(*args, noise=False, float_depth=True)
    noisy, _, _ = synth.render(*args, noise=True, dropout=0.02)
    return exact.astype(np.float64), noisy


def test_dropout_fraction():
    z, d = render_pair()
    # pixels whose noisy depth cannot leave the [0.3, 5] m window (|noise| < 5 sigma)
    inside = (z > 0.35) & (z < 4.5)
    frac = float((d[inside] == 0).mean())
    n = int(inside.sum())
    assert n > 400000
    assert abs(frac - 0.02) < 5 * np.sqrt(0.02 * 0.98 / n), frac


def test_axial_noise_variance_with_millimetre_rounding():
    z, d = render_pair()
    kept = (z > 0.35) & (z < 4.5) & (d > 0)
    zk, r = z[kept], d[kept].astype(np.float64) / 1000.0 - z[kept]
    edges = np.quantile(zk, [0.0, 0.25, 0.5, 0.75, 1.0])
    for lo, hi in zip(edges[:-1], edges[1:]):
        sel = (zk >= lo) & (zk < hi)
        n = int(sel.sum())
        assert n > 50000
        sig2 = np.mean((0.0012 + 0.0019 * (zk[sel] - 0.4) ** 2) ** 2) + 1e-6 / 12.0  # + rounding to 1 mm
        var = float(r[sel].var())
        assert abs(var / sig2 - 1.0) < 6 * np.sqrt(2.0 / n) + 0.01, (lo, hi, var, sig2)
        assert abs(float(r[sel].mean())) < 5 * np.sqrt(sig2 / n), (lo, hi)
