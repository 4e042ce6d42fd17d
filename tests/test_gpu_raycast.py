"""Virtual depth (raycast_depth, Sec. III-E) through the C ABI against the
oracle: bit-exact against the FP32 mirror on analytic maps and on a fused
map, close to the FP64 reference; the fill mode keeps valid depths; the
VirtualDepth helper refines the holes of real frames from an n-frame model."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from gpu_helpers import dev_pose, gpu_frame, map_params, need_gpu, orc_frame, oracle_maps
from synth import analytic as A

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rf():
    return need_gpu()


def import_both(rf, keys, sdf, w, rgb, s, tau):
    mp = rf.MapParams(s, tau, 5.0, 1 << 16, 1 << 15, 255, 4, "fp32", 64 * 64)
    m = rf.Map(mp)
    sdf32 = sdf.astype(np.float32)
    m.import_(torch.from_numpy(keys).cuda(), torch.from_numpy(sdf32).cuda(),
              torch.from_numpy(w.astype(np.float32)).cuda(), torch.from_numpy(rgb).cuda())
    oms = []
    for bits in (32, 64):
        o = O.OracleMap(s, tau, 5.0, 255, 4, real_bits=bits)
        o.import_(keys, sdf32.astype(np.float64), w, rgb)
        oms.append(o)
    return m, oms[0], oms[1]


def frames_for(rf, W, H, f, depth):
    g = rf.Frame(torch.from_numpy(depth).cuda(), torch.zeros((H, W, 3), dtype=torch.uint8, device="cuda"),
                 f, f, (W - 1) / 2.0, (H - 1) / 2.0, 1.0)
    o = O.Frame(depth, np.zeros((H, W, 3), np.uint8), f, f, (W - 1) / 2.0, (H - 1) / 2.0)
    return g, o


@pytest.mark.parametrize("shape", ["sphere", "plane"])
def test_raycast_of_analytic_map_matches_oracle(rf, shape):
    s, tau = 0.01, 0.05
    if shape == "sphere":
        c, r = np.array([0.05, -0.03, 1.2]), 0.3
        ang, pol = np.linspace(0, 2 * np.pi, 90), np.linspace(0, np.pi, 45)
        pts = c + r * np.array([[np.cos(a) * np.sin(b), np.sin(a) * np.sin(b), np.cos(b)] for a in ang for b in pol])
        keys = A.blocks_near(pts, s, 1)
        fn = lambda x: np.clip(np.linalg.norm(x - c, axis=-1) - r, -tau, tau)
    else:
        n = np.array([0.0, np.sin(0.3), np.cos(0.3)])
        B = 8 * s
        keys = np.array([[x, y, z] for x in range(-11, 11) for y in range(-9, 9) for z in range(10, 28)], np.int32)
        fn = lambda x: np.clip(1.4 - x @ n, -tau, tau)
    k, sdf, w, rgb = A.fill_map(keys, s, fn)
    m, o32, o64 = import_both(rf, k, sdf, w, rgb, s, tau)
    W, H = 64, 48
    g, o = frames_for(rf, W, H, 50.0, np.zeros((H, W), np.float32))
    T = np.eye(4)
    T[:3, 3] = [0.01, -0.02, 0.03]
    zg = m.raycast(g, dev_pose(T), only_invalid=False).cpu().numpy()
    z32 = o32.raycast(o, T, only_invalid=False)
    z64 = o64.raycast(o, T, only_invalid=False)
    assert (zg > 0).sum() > 500
    assert np.array_equal(zg, z32)                                # bit-exact vs the FP32 mirror
    both = (zg > 0) & (z64 > 0)
    assert both.sum() >= 0.99 * (zg > 0).sum()
    assert np.abs(zg[both] - z64[both]).max() < 1e-4              # FP64 reference


@pytest.mark.parametrize("storage,orc_storage", [("fp32", 0), ("fp16", 1)])
def test_raycast_of_fused_map_fills_holes_like_the_oracle(rf, storage, orc_storage):
    seq = synth.parity_room(n_frames=5)
    m = rf.Map(map_params(rf, seq, storage))
    o64, o32 = oracle_maps(seq, orc_storage)
    for k in range(4):
        g = gpu_frame(rf, seq, k)
        P = dev_pose(seq.poses[k])
        m.allocate(g, P)
        m.integrate(g, P)
        for o in (o64, o32):
            o.allocate(orc_frame(seq, k), seq.poses[k])
            o.integrate(orc_frame(seq, k), seq.poses[k])
    rng = np.random.default_rng(5)
    depth = seq.depth[4].copy()
    holes = rng.uniform(size=depth.shape) < 0.2
    depth[holes] = 0
    g = rf.Frame.from_numpy(depth, seq.rgb[4], *seq.intrinsics, depth_scale=seq.depth_scale)
    o = O.Frame(depth, seq.rgb[4], *seq.intrinsics, depth_scale=seq.depth_scale)
    zg = m.raycast(g, dev_pose(seq.poses[4]), far_value=4.0).cpu().numpy()
    z32 = o32.raycast(o, seq.poses[4], far_value=4.0)
    assert np.array_equal(zg, z32)
    truth = seq.depth[4].astype(np.float32) * np.float32(seq.depth_scale if seq.depth.dtype == np.uint16 else 1.0)
    keep = ~holes & (seq.depth[4] > 0)
    assert np.array_equal(zg[keep], truth[keep])                  # valid depths untouched
    filled = holes & (seq.depth[4] > 0) & (zg != 4.0)
    assert filled.sum() > 0.5 * holes.sum()
    assert np.median(np.abs(zg[filled] - truth[filled])) < 0.01   # the model explains the holes


def test_virtual_depth_helper_refines_holes(rf):
    seq = synth.dynamic_room(n_frames=6, width=160, height=120, n_clusters=1, movers="in_view")
    vd = rf.VirtualDepth(map_params(rf, seq), n=6, far_value=5.0)
    rng = np.random.default_rng(1)
    outs, holes = [], []
    for k in range(6):
        d = seq.depth[k].copy()
        h = rng.uniform(size=d.shape) < 0.15
        d[h] = 0
        holes.append(h & (seq.depth[k] > 0))
        outs = vd.push(rf.Frame.from_numpy(d, seq.rgb[k], *seq.intrinsics, depth_scale=seq.depth_scale),
                       dev_pose(seq.poses[k]))
        assert (len(outs) == 0) == (k < 5)
    assert len(outs) == 6
    errs = []
    for k, (f, P) in enumerate(outs):
        z = f.depth.cpu().numpy()
        truth = seq.depth[k].astype(np.float32) * np.float32(seq.depth_scale)
        sel = holes[k] & (z < 5.0)
        errs.append(np.abs(z[sel] - truth[sel]))
        assert (z[seq.depth[k] == 0] > 0).all()                    # no zero is left
    assert np.median(np.concatenate(errs)) < 0.01
