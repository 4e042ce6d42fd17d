"""Pins of the oracle's photometric term (Sec. III-B, Eqs. 3-4), its colour
running average (Sec. III-A) and its free-space carving in front of far
measurements (Sec. III-D) against closed forms (no GPU).

The photometric scene is a fronto-parallel plane z = c seen from the identity
pose whose voxel colours are affine in the voxel index (R = 128 + vx,
G = 128 + vy, B = 60): a trilinear interpolant reproduces affine fields
exactly, so the model intensity and its gradient at any point are known in
closed form, and the frame's pixels (one pixel per voxel on the plane) carry
exactly the model's colour at the true pose.
"""
import ctypes
import os
import subprocess
import tempfile
from fractions import Fraction

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import oracle as O
from synth import analytic as A

# luminance weights of Sec. III-B as the FP32 constants both implementations use
KR, KG, KB = (float(np.float32(x)) for x in (0.2126, 0.7152, 0.0722))


def luminance_ref(rgb):
    rgb = np.asarray(rgb, np.float64)
    return (KR * rgb[..., 0] + KG * rgb[..., 1] + KB * rgb[..., 2]) / 255.0


# --- the kernels' quotient: x / 255 without a division -----------------------

_QUOTIENT_C = r"""
#include <math.h>
#include <stdint.h>
/* For every RGB8 colour: x = (0.2126 R + 0.7152 G) + 0.0722 B in FP32;
   out[0] counts colours where x * RN(1/255) differs from the correctly
   rounded x / 255, out[1] those where the FMA-corrected quotient
   fma(fma(-q, 255, x), RN(1/255), q) differs from it. */
void check(int64_t* out) {
  const float r255 = 1.0f / 255.0f;
  out[0] = out[1] = 0;
  for (int R = 0; R < 256; ++R)
    for (int G = 0; G < 256; ++G)
      for (int B = 0; B < 256; ++B) {
        volatile float a = 0.2126f * (float)R, b = 0.7152f * (float)G, c = 0.0722f * (float)B;
        volatile float x = (a + b) + c;
        volatile float exact = x / 255.0f;
        volatile float q = x * r255;
        volatile float corrected = fmaf(fmaf(-q, 255.0f, x), r255, q);
        out[0] += (q != exact);
        out[1] += (corrected != exact);
      }
}
"""


def test_fma_corrected_quotient_is_the_correctly_rounded_division():
    """The kernels form I = x / 255 as one Newton correction of x * RN(1/255)
    (Markstein); over all 2^24 RGB8 colours it equals the correctly rounded
    division that the oracle's FP32 mirror performs (Sec. III-B intensity)."""
    with tempfile.TemporaryDirectory() as d:
        src, lib = os.path.join(d, "q.c"), os.path.join(d, "q.so")
        with open(src, "w") as fh:
            fh.write(_QUOTIENT_C)
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC", src,
                               "-o", lib, "-lm"])
        L = ctypes.CDLL(lib)
        out = np.zeros(2, np.int64)
        L.check(ctypes.c_void_p(out.ctypes.data))
    assert out[0] > 0, "the plain reciprocal product must differ somewhere (else the check is vacuous)"
    assert out[1] == 0


# --- model intensity of constant colours --------------------------------------

def plane_keys(s, c, half=0.4):
    xs = np.arange(-half, half + 1e-9, 4 * s)
    pts = np.array([[x, y, c] for x in xs for y in xs])
    return A.blocks_near(pts, s, 2)


@pytest.mark.parametrize("bits", [64, 32])
@pytest.mark.parametrize("rgb", [(255, 0, 0), (0, 255, 0), (0, 0, 255), (10, 200, 37), (255, 255, 255)])
def test_model_intensity_of_constant_colour(bits, rgb):
    """Iv of a map with one colour everywhere is (0.2126 R + 0.7152 G +
    0.0722 B) / 255 with zero gradient: pure red gives 0.2126, pure green
    0.7152, pure blue 0.0722, white 1."""
    s, c = 0.02, 1.0
    keys = plane_keys(s, c, 0.2)
    m = O.OracleMap(s, 0.1, real_bits=bits)
    m.import_(*A.fill_map(keys, s, lambda p: c - p[..., 2], lambda p: np.broadcast_to(np.float64(rgb), p.shape)))
    expect = (0.2126 * rgb[0] + 0.7152 * rgb[1] + 0.0722 * rgb[2]) / 255.0
    rng = np.random.default_rng(3)
    for _ in range(20):
        y = np.array([rng.uniform(-0.1, 0.1), rng.uniform(-0.1, 0.1), c + rng.uniform(-0.03, 0.03)])
        ok, out = m.sample(y)
        assert ok
        assert abs(out[4] - expect) < 2e-7, (out[4], expect)
        assert np.all(out[5:8] == 0.0)


# --- closed-form normal equations of the textured plane ----------------------

S_VOX, C_PLANE, F_PIX, C_PIX, N_PIX = 0.01, 1.0, 100.0, 20.0, 40


def plane_colour(vx, vy, split):
    """RGB of voxel (vx, vy) on the plane: affine R = 128 + vx, G = 128 + vy,
    B = 60; with split, R = 128 + min(vx, 0) and G = 128 + vy only where
    vx >= 0 (G = 128 elsewhere), so the intensity gradient points along x on
    the left half and along y on the right half."""
    if not split:
        return np.stack([128 + vx, 128 + vy, np.full(np.shape(vx), 60.0)], -1)
    return np.stack([128 + np.minimum(vx, 0), np.where(vx >= 0, 128 + vy, 128), np.full(np.shape(vx), 60.0)], -1)


def textured_plane(bits=64, tau=0.05, split=False):
    """Map of the plane z = C_PLANE (sdf = c - z) with the colours of
    plane_colour, and the 40x40 frame of it from the identity pose: depth c,
    pixel (u, v) sees voxel (u - 20, v - 20) and carries its colour (with
    split: the pixels whose cells could straddle vx = 0 have no depth)."""
    s = S_VOX
    sf = float(np.float32(s))
    keys = plane_keys(s, C_PLANE, 0.4)
    m = O.OracleMap(s, tau, real_bits=bits)
    m.import_(*A.fill_map(keys, s, lambda p: C_PLANE - p[..., 2],
                          lambda p: plane_colour(np.rint(p[..., 0] / sf), np.rint(p[..., 1] / sf), split)))
    u, v = np.meshgrid(np.arange(N_PIX), np.arange(N_PIX))
    rgb = plane_colour(u - 20, v - 20, split).astype(np.uint8)
    depth = np.full((N_PIX, N_PIX), C_PLANE, np.float32)
    if split:
        depth[:, 16:25] = 0.0
    fr = O.Frame(depth, rgb, F_PIX, F_PIX, C_PIX, C_PIX)
    return m, fr, depth, rgb


def closed_form_normal_equations(T, depth, rgb, level, w_c):
    """H, g, cost, count of Eq. 4 from the closed forms: S(y) = c - y_z,
    grad S = (0, 0, -1); Iv(y) = (KR (128 + y_x/s) + KG (128 + y_y/s) + KB 60)/255,
    grad Iv = (KR, KG, 0) / (255 s); J = [grad, y x grad]; r_c = Iv(y) - I(p)."""
    sf = float(np.float32(S_VOX))
    st = 1 << level
    H = np.zeros((6, 6))
    g = np.zeros(6)
    cost = 0.0
    n = 0
    gS = np.array([0.0, 0.0, -1.0])
    gI = np.array([KR, KG, 0.0]) / (255.0 * sf)
    for v in range(0, depth.shape[0], st):
        for u in range(0, depth.shape[1], st):
            D = float(depth[v, u])
            x = np.array([(u - C_PIX) / F_PIX * D, (v - C_PIX) / F_PIX * D, D])
            y = T[:3, :3] @ x + T[:3, 3]
            S = C_PLANE - y[2]
            Iv = (KR * (128 + y[0] / sf) + KG * (128 + y[1] / sf) + KB * 60) / 255.0
            rc = Iv - luminance_ref(rgb[v, u])
            Jd = np.r_[gS, np.cross(y, gS)]
            Jc = np.r_[gI, np.cross(y, gI)]
            H += np.outer(Jd, Jd) + w_c * np.outer(Jc, Jc)
            g += Jd * S + w_c * Jc * rc
            cost += S * S + w_c * rc * rc
            n += 1
    return H, g, cost, n


@pytest.mark.parametrize("w_c", [0.025, 1.0])
@pytest.mark.parametrize("level", [0, 1])
def test_normal_equations_carry_the_photometric_term(w_c, level):
    """Eq. 4: H = sum J_d^T J_d + w_c J_c^T J_c, g = sum J_d^T r_d + w_c J_c^T r_c,
    cost = sum r_d^2 + w_c r_c^2, against the closed forms of the textured
    plane at a pose off the truth (so S and r_c are non-zero)."""
    m, fr, depth, rgb = textured_plane()
    T = O.pose_left_update(np.r_[0.012, -0.007, 0.006, 0.01, -0.015, 0.02], np.eye(4))
    ne = m.normal_equations(fr, T, level=level, w_c=w_c)
    H, g, cost, n = closed_form_normal_equations(T, depth, rgb, level, w_c)
    assert ne[28] == n == (N_PIX >> level) ** 2
    iu = np.triu_indices(6)
    np.testing.assert_allclose(ne[:21], H[iu], rtol=1e-9, atol=1e-9 * np.abs(H).max())
    np.testing.assert_allclose(ne[21:27], g, rtol=1e-9, atol=1e-9 * np.abs(g).max())
    assert abs(ne[27] - cost) <= 1e-9 * cost
    # the in-plane translation rows come from the photometric term alone
    assert H[0, 0] > 0 and abs(H[0, 0] - w_c * n * (KR / (255.0 * float(np.float32(S_VOX)))) ** 2) <= 1e-9 * H[0, 0]


def test_photometric_term_makes_the_in_plane_motion_observable():
    """A plane's SDF leaves the in-plane translations and the rotation about
    its normal unconstrained: with w_c = 0 the system is singular and the pass
    stops with the pose kept; with w_c > 0 (Table I: 0.025) the texture
    (intensity gradients along x on one half of the plane and along y on the
    other, each half exactly affine) recovers a known in-plane shift and
    rotation exactly, since every residual vanishes at the true pose."""
    m, fr, depth, rgb = textured_plane(split=True)
    rng = np.random.default_rng(14)
    for _ in range(3):
        xi = np.r_[rng.uniform(-0.01, 0.01, 2), rng.uniform(-0.005, 0.005), np.radians(rng.uniform(-0.3, 0.3, 2)),
                   np.radians(rng.uniform(-0.5, 0.5))]
        T0 = O.pose_left_update(xi, np.eye(4))
        T, flags, _ = m.track(fr, T0, levels=2, iters=10, w_c=0.025)
        assert flags == 0
        assert np.linalg.norm(T[:3, 3]) < 1e-6
        assert np.linalg.norm(Rotation.from_matrix(T[:3, :3]).as_rotvec()) < 1e-6
        T, flags, _ = m.track(fr, T0, levels=2, iters=10, w_c=0.0)
        assert flags & 2 and np.array_equal(T, T0)


def test_fp32_mirror_photometric_normal_equations_match_fp64():
    m64, fr, depth, rgb = textured_plane(64)
    m32, _, _, _ = textured_plane(32)
    T = O.pose_left_update(np.r_[0.01, 0.004, -0.003, 0.0, 0.01, -0.02], np.eye(4))
    a = m64.normal_equations(fr, T, 0, 1.0)
    b = m32.normal_equations(fr, T, 0, 1.0)
    assert a[28] == b[28]
    np.testing.assert_allclose(b[:28], a[:28], rtol=1e-4, atol=1e-4 * np.abs(a[:21]).max())


# --- colour running average (Sec. III-A), rounded half to even ----------------

def rhe_average(W, C, c):
    """round_half_even((W C + c) / (W + 1)) in exact rational arithmetic."""
    q = Fraction(W * C + c, W + 1)
    fl = q.numerator // q.denominator
    rem = q - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return fl


@pytest.mark.parametrize("bits", [64, 32])
@pytest.mark.parametrize("w_max", [255, 3])
def test_colour_running_average_rounds_half_to_even(bits, w_max):
    """Band voxels average the colour with the same weights as the sdf and
    store RGB8 rounded half to even; the sequence is chosen so that exact .5
    ties occur (frame 2: 10.5 -> 10, 21.5 -> 22, 35.5 -> 36; with W capped at
    3 also (3 C + c) / 4 ties)."""
    s, tau, d = 0.02, 0.06, 0.71
    cols = [(10, 20, 31), (11, 23, 40), (12, 0, 9), (12, 22, 41), (200, 7, 100), (13, 22, 38), (0, 255, 3)]
    m = O.OracleMap(s, tau, 5.0, w_max, 2, real_bits=bits)
    for col in cols:
        fr = O.Frame(np.full((30, 40), d, np.float32), np.broadcast_to(np.uint8(col), (30, 40, 3)).copy(),
                     30.0, 30.0, 19.5, 14.5)
        m.allocate(fr, np.eye(4))
        m.integrate(fr, np.eye(4))
    keys, sdf, w, rgb = m.export()
    c = A.block_voxel_centres(keys, s).reshape(-1, 3)
    rgb = rgb.reshape(-1, 3)
    w = w.reshape(-1)
    z = c[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = np.floor(30.0 * (c[:, 0] / z) + 19.5 + 0.5)
        v = np.floor(30.0 * (c[:, 1] / z) + 14.5 + 0.5)
    inside = (z > 0) & (u >= 0) & (u < 40) & (v >= 0) & (v < 30)
    band = inside & (np.abs(float(np.float32(d)) - z) <= tau - 1e-6)
    assert band.sum() > 100
    expect = np.zeros(3, np.int64)
    W = 0
    ties = 0
    for col in cols:
        for k in range(3):
            ties += (W * int(expect[k]) + col[k]) * 2 % (W + 1) == 0 and (W * int(expect[k]) + col[k]) % (W + 1) != 0
            expect[k] = rhe_average(W, int(expect[k]), col[k])
        W = min(W + 1, w_max)
    assert ties >= 3
    assert np.all(rgb[band] == expect), (np.unique(rgb[band], axis=0), expect)
    assert np.all(w[band] == min(len(cols), w_max))


# --- free space in front of measurements beyond depth_max (Sec. III-D) --------

@pytest.mark.parametrize("bits", [64, 32])
def test_far_measurement_carves_up_to_the_clipping_plane(bits):
    """A wall at 3 m with depth_max = 1.5 m: no band voxel is integrated, and
    every visited voxel in the view with 0 < z <= 1.5 m is carved to tau once,
    those beyond the clipping plane stay unobserved; allocation walks the
    carve segments [0, depth_max] only."""
    s, tau, zclip, d = 0.05, 0.15, 1.5, 3.0
    W, H, f = 24, 18, 20.0
    m = O.OracleMap(s, tau, zclip, 255, 1, real_bits=bits)
    fr = O.Frame(np.full((H, W), d, np.float32), np.full((H, W, 3), 77, np.uint8), f, f, (W - 1) / 2, (H - 1) / 2)
    keys = m.allocate(fr, np.eye(4))
    B = 8 * float(np.float32(s))
    assert len(keys) > 0 and keys[:, 2].min() * B < 0.01 and keys[:, 2].max() * B <= zclip
    counts = m.integrate(fr, np.eye(4))
    assert counts[0] == 0 and counts[1] > 0
    k2, sdf, w, rgb = m.export()
    c = A.block_voxel_centres(k2, s).reshape(-1, 3)
    sdf, w = sdf.reshape(-1), w.reshape(-1)
    z = c[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = np.floor(f * (c[:, 0] / z) + (W - 1) / 2 + 0.5)
        v = np.floor(f * (c[:, 1] / z) + (H - 1) / 2 + 0.5)
    inside = (z > 0) & (u >= 0) & (u < W) & (v >= 0) & (v < H)
    carved = inside & (z <= zclip - 1e-6)
    beyond = ~inside | (z > zclip + 1e-6)
    assert carved.sum() > 100
    np.testing.assert_allclose(sdf[carved], float(np.float32(tau)), rtol=0, atol=1e-7)
    assert np.all(w[carved] == 1)
    assert np.all(w[beyond] == 0)
    assert counts[1] == int((w == 1).sum())
    assert np.all(inside[w == 1] & (z[w == 1] <= zclip + 1e-6))
    # the same wall within depth_max is integrated in its band as before
    m2 = O.OracleMap(s, tau, 5.0, 255, 1, real_bits=bits)
    m2.allocate(fr, np.eye(4))
    assert m2.integrate(fr, np.eye(4))[0] > 0


def test_far_measurements_are_not_registered():
    """Registration uses valid pixels only (0 < D <= depth_max): pushing part
    of a frame beyond depth_max removes exactly those pixels from the count."""
    m, fr, depth, rgb = textured_plane()
    T = np.eye(4)
    n_all = m.normal_equations(fr, T, 0, 0.025)[28]
    d2 = depth.copy()
    d2[:, :10] = 9.0
    fr2 = O.Frame(d2, rgb, F_PIX, F_PIX, C_PIX, C_PIX)
    assert m.normal_equations(fr2, T, 0, 0.025)[28] == n_all - 10 * N_PIX
