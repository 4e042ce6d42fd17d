"""Pins of the CPU oracle against mathematics, closed forms and library
routines (no GPU).  Each test names the passage of the paper it pins."""
import itertools
import math

import numpy as np
import pytest
import scipy.linalg
import scipy.ndimage
from scipy.spatial.transform import Rotation

import oracle as O
import synth
from synth import analytic as A


def twist_matrix(xi):
    rho, phi = xi[:3], xi[3:]
    M = np.zeros((4, 4))
    M[:3, :3] = [[0, -phi[2], phi[1]], [phi[2], 0, -phi[0]], [-phi[1], phi[0], 0]]
    M[:3, 3] = rho
    return M


# --- Section III-B: exponential map of se(3) -------------------------------

def test_exp_zero_is_identity():
    assert np.array_equal(O.se3_exp(np.zeros(6)), np.eye(4))


@pytest.mark.parametrize("scale", [1e-9, 1e-6, 1e-3, 5e-3, 0.02, 0.3, 1.0, 2.5])
def test_exp_matches_matrix_exponential(scale):
    rng = np.random.default_rng(int(scale * 1e9) % 2**32)
    for _ in range(20):
        xi = rng.normal(size=6) * scale
        ref = scipy.linalg.expm(twist_matrix(xi))
        np.testing.assert_allclose(O.se3_exp(xi), ref, rtol=0, atol=2e-14 * max(1.0, scale) ** 2)


def test_exp_pure_rotation_and_translation():
    rng = np.random.default_rng(3)
    for _ in range(10):
        phi = rng.normal(size=3)
        T = O.se3_exp(np.r_[0, 0, 0, phi])
        np.testing.assert_allclose(T[:3, :3], Rotation.from_rotvec(phi).as_matrix(), atol=1e-14)
        np.testing.assert_allclose(T[:3, 3], 0, atol=0)
        rho = rng.normal(size=3)
        T = O.se3_exp(np.r_[rho, 0, 0, 0])
        np.testing.assert_allclose(T[:3, :3], np.eye(3), atol=0)
        np.testing.assert_allclose(T[:3, 3], rho, atol=1e-15)


def test_log_of_exp_roundtrip():
    rng = np.random.default_rng(4)
    for _ in range(10):
        xi = rng.normal(size=6) * 0.4
        L = scipy.linalg.logm(O.se3_exp(xi)).real
        np.testing.assert_allclose(L, twist_matrix(xi), atol=1e-12)


def test_left_update_composes_on_the_left():
    rng = np.random.default_rng(5)
    T = O.se3_exp(rng.normal(size=6))
    xi = rng.normal(size=6) * 0.1
    np.testing.assert_allclose(O.pose_left_update(xi, T), scipy.linalg.expm(twist_matrix(xi)) @ T, atol=1e-13)


# --- FP16 storage rounding (precision form) against numpy's binary16 --------

def test_round_to_half_matches_numpy_float16():
    rng = np.random.default_rng(6)
    xs = np.concatenate([rng.uniform(-1.5, 1.5, 4000), rng.normal(size=2000) * 1e-5,
                         rng.uniform(-70000, 70000, 500)]).astype(np.float32)
    # exact ties: halfway between consecutive binary16 values
    h = rng.uniform(-1, 1, 500).astype(np.float16)
    nxt = np.nextafter(h, np.float16(np.inf))
    ties = ((h.astype(np.float64) + nxt.astype(np.float64)) / 2).astype(np.float32)
    for x in np.concatenate([xs, ties, np.float32([0.0, -0.0, 6.1e-5, 5.96e-8, 65504.0, 65519.0, 65520.0])]):
        with np.errstate(over="ignore"):
            ref = np.float32(np.float16(x))
        got = O.round_to_half(x)
        assert got == ref or (np.isinf(ref) and np.isinf(got)), (x, got, ref)


# --- Section III-B: trilinear interpolation of the voxel field ---------------

def affine_map(voxel, a, c0):
    keys = np.array(list(itertools.product(range(-1, 2), repeat=3)), np.int32)
    return A.fill_map(keys, voxel, lambda p: p @ np.asarray(a) + c0)


def test_trilinear_reproduces_affine_fields_exactly():
    s = 0.02
    a, c0 = np.array([0.3, -0.7, 0.45]), 0.011
    m = O.OracleMap(s, 10.0, real_bits=64)
    m.import_(*affine_map(s, a, c0))
    rng = np.random.default_rng(7)
    B = 8 * float(np.float32(s))
    for y in rng.uniform(-B + 0.01, B * 2 - 0.05, size=(200, 3)):
        ok, out = m.sample(y)
        assert ok
        assert abs(out[0] - (a @ y + c0)) < 1e-14
        np.testing.assert_allclose(out[1:4], a, atol=1e-11)


def test_trilinear_equals_eight_weight_formula():
    s = float(np.float32(0.05))
    rng = np.random.default_rng(8)
    keys = np.zeros((1, 3), np.int32)
    vals = rng.normal(size=(1, 512))
    m = O.OracleMap(s, 100.0, real_bits=64)
    m.import_(keys, vals, np.ones((1, 512)), np.full((1, 512, 3), 100, np.uint8))
    V = vals.reshape(8, 8, 8)  # [lz, ly, lx]
    for _ in range(200):
        g = rng.uniform(0, 6.999, 3)
        i0 = np.floor(g).astype(int)
        f = g - i0
        ref = 0.0
        for dx, dy, dz in itertools.product((0, 1), repeat=3):
            wgt = (f[0] if dx else 1 - f[0]) * (f[1] if dy else 1 - f[1]) * (f[2] if dz else 1 - f[2])
            ref += wgt * V[i0[2] + dz, i0[1] + dy, i0[0] + dx]
        ok, out = m.sample(g * s)
        assert ok
        assert abs(out[0] - ref) < 1e-12


def test_sample_undefined_without_eight_observed_corners():
    s = 0.02
    keys, sdf, w, rgb = affine_map(s, [1, 0, 0], 0)
    w[13, 0] = 0.0  # the voxel (0,0,0) of block (0,0,0) unobserved
    m = O.OracleMap(s, 10.0, real_bits=64)
    m.import_(keys, sdf, w, rgb)
    assert not m.sample(np.array([0.5, 0.5, 0.5]) * s)[0]
    assert not m.sample(np.array([-0.5, -0.5, -0.5]) * s)[0]
    assert m.sample(np.array([1.5, 0.5, 0.5]) * s)[0]
    assert not m.sample(np.array([100.0, 0, 0]))[0]   # no block there


# --- Eqs. (2)-(4): analytic Jacobians vs central finite differences ---------

def smooth_map(s, tau):
    centre = np.array([0.05, -0.02, 0.8])
    pts = centre + np.array(list(itertools.product([-0.3, 0, 0.3], repeat=3)))
    keys = A.blocks_near(pts, s, 2)
    return A.fill_map(keys, s, lambda p: np.linalg.norm(p - centre, axis=-1) - 0.25,
                      lambda p: np.repeat((128 + 90 * np.sin(7 * p[..., :1]) * np.cos(5 * p[..., 1:2])
                                           + 30 * np.sin(9 * p[..., 2:3])), 3, -1))


def test_jacobian_matches_central_differences():
    s, tau = 0.02, 0.2
    m = O.OracleMap(s, tau, real_bits=64)
    m.import_(*smooth_map(s, tau))
    rng = np.random.default_rng(9)
    T = O.se3_exp(np.r_[0.01, -0.02, 0.03, 0.02, -0.01, 0.015])
    h = 1e-6
    checked = 0
    for _ in range(400):
        x = np.array([rng.uniform(-0.3, 0.3), rng.uniform(-0.3, 0.3), 0.55 + rng.uniform(0, 0.05)])
        y = T[:3, :3] @ x + T[:3, 3]
        f = y / float(np.float32(s))
        fr = f - np.floor(f)
        if np.any(fr < 0.02) or np.any(fr > 0.98):
            continue
        ok, t0 = m.pixel_terms(x, T, 0.4)
        if not ok:
            continue
        for k in range(6):
            e = np.zeros(6)
            e[k] = h
            okp, tp = m.pixel_terms(x, O.pose_left_update(e, T), 0.4)
            okm, tm = m.pixel_terms(x, O.pose_left_update(-e, T), 0.4)
            assert okp and okm
            fd_d = (tp[0] - tm[0]) / (2 * h)
            fd_c = (tp[7] - tm[7]) / (2 * h)
            assert abs(fd_d - t0[1 + k]) <= 1e-6 * max(1.0, abs(t0[1 + k])), (k, fd_d, t0[1 + k])
            assert abs(fd_c - t0[8 + k]) <= 1e-6 * max(1.0, abs(t0[8 + k])), (k, fd_c, t0[8 + k])
        checked += 1
    assert checked > 50


# --- Section III-B: normal equations and solve --------------------------------

def unpack_H(ne):
    H = np.zeros((6, 6))
    iu = np.triu_indices(6)
    H[iu] = ne[:21]
    H = H + H.T - np.diag(np.diag(H))
    return H


def test_normal_equations_symmetric_psd_full_rank(parity_seq):
    s = parity_seq
    m = O.OracleMap(s.voxel_size, s.truncation, s.depth_max, 255, s.carve_stride)
    fr = O.Frame(s.depth[0], s.rgb[0], *s.intrinsics)
    m.allocate(fr, s.poses[0])
    m.integrate(fr, s.poses[0])
    fr1 = O.Frame(s.depth[1], s.rgb[1], *s.intrinsics)
    for level in (0, 1):
        ne = m.normal_equations(fr1, s.poses[0], level)
        H = unpack_H(ne)
        ev = np.linalg.eigvalsh(H)
        assert ev.min() > 1e-9 * np.trace(H)
        assert ne[28] > 1000 and ne[27] > 0
        # H = sum of outer products => g lies in its range; cost >= g^T H^-1 g
        gv = ne[21:27]
        assert gv @ np.linalg.solve(H, gv) <= ne[27] * (1 + 1e-9)


def test_solve6_matches_numpy_and_flags_singular():
    rng = np.random.default_rng(10)
    for _ in range(20):
        J = rng.normal(size=(50, 6))
        H = J.T @ J
        g = rng.normal(size=6)
        ne = np.r_[H[np.triu_indices(6)], g, 0.0, 50.0]
        np.testing.assert_allclose(O.solve6(ne), np.linalg.solve(H, -g), rtol=1e-10, atol=1e-12)
        lam = 0.3
        np.testing.assert_allclose(O.solve6(ne, lam), np.linalg.solve(H + lam * np.diag(np.diag(H)), -g),
                                   rtol=1e-10, atol=1e-12)
    J = rng.normal(size=(50, 5)) @ rng.normal(size=(5, 6))   # rank 5
    ne = np.r_[(J.T @ J)[np.triu_indices(6)], np.ones(6), 0.0, 50.0]
    assert O.solve6(ne) is None


def corner_scene(voxel=0.01, tau=0.1, W=160, H=120, f=120.0, margin_vox=4):
    """Room corner x, y, z >= 0 with the exact SDF min(x, y, z) in the map and
    a depth image of the three planes seen from inside; pixels whose point is
    within margin_vox voxels of an edge are dropped (depth 0)."""
    pose = np.eye(4)
    o = np.array([0.55, 0.5, 0.6])
    fwd = -o / np.linalg.norm(o)
    r = np.cross(fwd, [0.0, 0.0, 1.0]); r /= np.linalg.norm(r)
    d = np.cross(fwd, r)
    pose[:3, 0], pose[:3, 1], pose[:3, 2], pose[:3, 3] = r, d, fwd, o
    cx, cy = (W - 1) / 2, (H - 1) / 2
    planes = [((1, 0, 0), 0.0), ((0, 1, 0), 0.0), ((0, 0, 1), 0.0)]
    z, pts, idx = A.ray_depth_planes(pose, W, H, f, f, cx, cy, planes)
    srt = np.sort(pts, axis=-1)
    keep = (idx >= 0) & (srt[..., 1] > margin_vox * voxel) & (srt[..., 0] > -1e-9)
    depth = np.where(keep, z, 0).astype(np.float32)
    surf = pts[keep]
    keys = A.blocks_near(surf, voxel, 2)
    mp = A.fill_map(keys, voxel, lambda p: np.min(p, axis=-1))
    rgb = np.full((H, W, 3), 128, np.uint8)
    return pose, depth, rgb, mp, (f, f, cx, cy)


def test_tracking_recovers_known_rigid_transform():
    pose, depth, rgb, mp, K = corner_scene()
    m = O.OracleMap(0.01, 0.1, real_bits=64)
    m.import_(*mp)
    fr = O.Frame(depth, rgb, *K)
    rng = np.random.default_rng(11)
    for _ in range(3):
        xi = np.r_[rng.uniform(-0.03, 0.03, 3), np.radians(rng.uniform(-2, 2, 3))]
        T0 = O.pose_left_update(xi, pose)
        T, flags, st = m.track(fr, T0, levels=3, iters=15, w_c=0.0)
        assert flags == 0
        E = np.linalg.inv(pose) @ T
        assert np.linalg.norm(E[:3, 3]) < 1e-6
        assert np.linalg.norm(Rotation.from_matrix(E[:3, :3]).as_rotvec()) < 1e-6


# --- Levenberg-Marquardt variant (the solver Section III-B names) --------------

def test_lm_recovers_known_rigid_transform():
    pose, depth, rgb, mp, K = corner_scene()
    m = O.OracleMap(0.01, 0.1, real_bits=64)
    m.import_(*mp)
    fr = O.Frame(depth, rgb, *K)
    rng = np.random.default_rng(12)
    for _ in range(3):
        xi = np.r_[rng.uniform(-0.03, 0.03, 3), np.radians(rng.uniform(-2, 2, 3))]
        T, flags, st, trace = m.track_lm(fr, O.pose_left_update(xi, pose), levels=3, iters=15, w_c=0.0)
        assert flags == 0
        E = np.linalg.inv(pose) @ T
        assert np.linalg.norm(E[:3, 3]) < 1e-6
        assert np.linalg.norm(Rotation.from_matrix(E[:3, :3]).as_rotvec()) < 1e-6


def test_lm_with_zero_lambda_takes_the_gauss_newton_step():
    """lambda = 0: the first step is the Gauss-Newton step, so after one
    accepted step LM and GN return the same pose."""
    pose, depth, rgb, mp, K = corner_scene()
    m = O.OracleMap(0.01, 0.1, real_bits=64)
    m.import_(*mp)
    fr = O.Frame(depth, rgb, *K)
    T0 = O.pose_left_update(np.r_[0.01, -0.02, 0.015, 0.01, -0.02, 0.015], pose)
    T_gn, _, _ = m.track(fr, T0, levels=1, iters=1, w_c=0.0)
    T_lm, flags, st, trace = m.track_lm(fr, T0, levels=1, iters=2, w_c=0.0, lambda0=0.0)
    assert flags == 0 and trace[1, 3] == 1.0
    assert np.array_equal(T_lm, T_gn)


def test_lm_step_solves_the_damped_system():
    """With a large lambda the accepted step is delta = -(H + lambda diag H)^-1 g
    from the normal equations at the start pose (solved here with numpy)."""
    pose, depth, rgb, mp, K = corner_scene()
    m = O.OracleMap(0.01, 0.1, real_bits=64)
    m.import_(*mp)
    fr = O.Frame(depth, rgb, *K)
    T0 = O.pose_left_update(np.r_[0.02, 0.01, -0.01, 0.0, 0.02, 0.0], pose)
    lam = 50.0
    ne = m.normal_equations(fr, T0, level=0, w_c=0.0)
    H = np.zeros((6, 6))
    H[np.triu_indices(6)] = ne[:21]
    H = H + np.triu(H, 1).T
    delta = np.linalg.solve(H + lam * np.diag(np.diag(H)), -ne[21:27])
    T_lm, flags, st, trace = m.track_lm(fr, T0, levels=1, iters=2, w_c=0.0, lambda0=lam)
    assert flags == 0 and trace[1, 3] == 1.0 and trace[1, 1] < trace[0, 1]
    np.testing.assert_allclose(T_lm, O.pose_left_update(delta, T0), rtol=0, atol=1e-12)


def test_lm_never_returns_a_rejected_candidate():
    """Once converged, candidates whose mean cost is not lower are rejected; a
    rejected evaluation leaves the result unchanged (the run with one
    evaluation less returns the same pose), an accepted one moves it, and
    within a level the accepted mean cost never rises."""
    seq = synth.parity_room(n_frames=3)
    m = O.OracleMap(seq.voxel_size, seq.truncation, seq.depth_max, 255, seq.carve_stride, real_bits=64)
    for k in range(2):
        fr = O.Frame(seq.depth[k], seq.rgb[k], *seq.intrinsics)
        m.allocate(fr, seq.poses[k])
        m.integrate(fr, seq.poses[k])
    fr2 = O.Frame(seq.depth[2], seq.rgb[2], *seq.intrinsics)
    T0 = O.pose_left_update(np.r_[0.02, -0.02, 0.015, 0.03, -0.02, 0.04], seq.poses[2])
    n = 10
    _, _, _, trace = m.track_lm(fr2, T0, levels=1, iters=n, lambda0=0.0)
    acc = trace[:, 3] == 1
    assert acc[0] and not acc.all(), "the case must contain a rejection"
    costs = trace[acc, 1]
    assert np.all(np.diff(costs) <= 0)
    for e in range(1, n):
        T_e, _, _, _ = m.track_lm(fr2, T0, levels=1, iters=e + 1, lambda0=0.0)
        T_p, _, _, _ = m.track_lm(fr2, T0, levels=1, iters=e, lambda0=0.0)
        assert np.array_equal(T_e, T_p) == (not acc[e]), e


def test_tracking_flags_too_few_pixels():
    pose, depth, rgb, mp, K = corner_scene()
    m = O.OracleMap(0.01, 0.1, real_bits=64)
    m.import_(*mp)
    fr = O.Frame(np.zeros_like(depth), rgb, *K)
    T, flags, st = m.track(fr, pose, levels=2, iters=3)
    assert flags & 1 and np.array_equal(T, pose)


# --- Sections III-A/III-D: integration closed forms ---------------------------

def plane_frame(d, W=40, H=30, f=30.0, color=(200, 100, 50)):
    depth = np.full((H, W), d, np.float32)
    rgb = np.zeros((H, W, 3), np.uint8)
    rgb[:] = color
    return O.Frame(depth, rgb, f, f, (W - 1) / 2, (H - 1) / 2)


def voxel_table(m, s):
    keys, sdf, w, rgb = m.export()
    c = A.block_voxel_centres(keys, s).reshape(-1, 3)
    return c, sdf.reshape(-1), w.reshape(-1), rgb.reshape(-1, 3)


def projects_inside(c, W, H, f):
    z = c[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = np.floor(f * (c[:, 0] / z) + (W - 1) / 2 + 0.5)
        v = np.floor(f * (c[:, 1] / z) + (H - 1) / 2 + 0.5)
    return (z > 0) & (u >= 0) & (u < W) & (v >= 0) & (v < H)


@pytest.mark.parametrize("bits", [64, 32])
def test_fronto_parallel_plane_closed_form(bits):
    s, tau, d = 0.02, 0.06, 0.71
    m = O.OracleMap(s, tau, 5.0, 255, 2, real_bits=bits)
    fr = plane_frame(d)
    m.allocate(fr, np.eye(4))
    counts = m.integrate(fr, np.eye(4))
    c, sdf, w, rgb = voxel_table(m, s)
    D = float(np.float32(d))
    inside = projects_inside(c, 40, 30, 30.0)
    eta = D - c[:, 2]
    band = inside & (np.abs(eta) <= tau - 1e-6)
    free = inside & (eta > tau + 1e-6)
    occl = inside & (eta < -tau - 1e-6)
    tol = 1e-12 if bits == 64 else 1e-6
    assert band.sum() > 100 and free.sum() > 100 and occl.sum() > 10
    np.testing.assert_allclose(sdf[band], eta[band], atol=tol)
    assert np.all(w[band] == 1) and np.all(rgb[band] == [200, 100, 50])
    np.testing.assert_allclose(sdf[free], tau, atol=1e-7)
    assert np.all(w[free] == 1) and np.all(rgb[free] == 0)
    assert np.all(w[occl] == 0) and np.all(sdf[occl] == 0)
    assert counts[0] == np.sum(w > 0) - counts[1]


def test_two_planes_average_and_weight_cap():
    s, tau = 0.02, 0.06
    d1, d2 = 0.70, 0.73
    m = O.OracleMap(s, tau, 5.0, 3, 2)
    for d in (d1, d2, d1, d2, d1):
        fr = plane_frame(d, color=(10, 20, 30) if d == d1 else (20, 40, 61))
        m.allocate(fr, np.eye(4))
        m.integrate(fr, np.eye(4))
    c, sdf, w, rgb = voxel_table(m, s)
    inside = projects_inside(c, 40, 30, 30.0)
    e1 = float(np.float32(d1)) - c[:, 2]
    e2 = float(np.float32(d2)) - c[:, 2]
    both = inside & (np.abs(e1) < tau - 1e-6) & (np.abs(e2) < tau - 1e-6)
    assert both.sum() > 50
    # running average with weight capped at 3: W=0,1,2 plain mean, then W=3 fixed
    ref = e1.copy()
    for k, e in enumerate([e2, e1, e2, e1][:4], start=1):
        Wk = min(k, 3)
        ref = (Wk * ref + e) / (Wk + 1)
    np.testing.assert_allclose(sdf[both], ref[both], atol=1e-12)
    assert np.all(w[both] == 3)


def test_moved_object_decays_toward_truncation():
    """Section III-D: a plane that moves away is averaged toward tau."""
    s, tau = 0.02, 0.06
    m = O.OracleMap(s, tau, 5.0, 255, 1)
    for _ in range(4):
        fr = plane_frame(0.6)
        m.allocate(fr, np.eye(4)); m.integrate(fr, np.eye(4))
    c, sdf0, w0, _ = voxel_table(m, s)
    for _ in range(6):
        fr = plane_frame(1.2)
        m.allocate(fr, np.eye(4)); m.integrate(fr, np.eye(4))
    keys1, _, _, _ = m.export()
    c1, sdf1, w1, _ = voxel_table(m, s)
    inside = projects_inside(c1, 40, 30, 30.0)
    old = {tuple(np.round(p, 6)): (a, b) for p, a, b in zip(c, sdf0, w0)}
    checked = 0
    for p, a, b in zip(c1[inside], sdf1[inside], w1[inside]):
        key = tuple(np.round(p, 6))
        if key not in old or old[key][1] != 4 or p[2] > 1.2 - tau - 1e-6:
            continue
        x = old[key][0]
        for k in range(4, 10):
            x = (k * x + float(np.float32(tau))) / (k + 1)
        assert abs(a - x) < 1e-12 and b == 10
        checked += 1
    assert checked > 50


def test_sphere_zero_crossing_on_central_ray():
    s, tau = 0.01, 0.04
    W = H = 41
    f = 40.0
    c, R = 0.9, 0.25
    z = A.ray_depth_sphere(np.eye(4), W, H, f, f, 20.0, 20.0, (0, 0, c), R, background=3.0)
    fr = O.Frame(z.astype(np.float32), np.full((H, W, 3), 90, np.uint8), f, f, 20.0, 20.0)
    m = O.OracleMap(s, tau, 5.0, 255, 4)
    m.allocate(fr, np.eye(4))
    m.integrate(fr, np.eye(4))
    pts = m.surface()
    axial = pts[(np.abs(pts[:, 0]) < 1e-9) & (np.abs(pts[:, 1]) < 1e-9) & (pts[:, 6] == 2)]
    assert len(axial) == 1
    assert abs(axial[0, 2] - float(np.float32(c - R))) < 1e-9


# --- Section III-C: dynamics mask ----------------------------------------------

def brute_closure(seeds, D, theta):
    H, W = seeds.shape
    n = H * W
    adj = np.zeros((n, n), bool)
    for v, u in itertools.product(range(H), range(W)):
        p = v * W + u
        for dv, du in itertools.product((-1, 0, 1), repeat=2):
            if (du or dv) and 0 <= u + du < W and 0 <= v + dv < H:
                q = (v + dv) * W + u + du
                adj[p, q] = abs(np.float32(D[v, u]) - np.float32(D[v + dv, u + du])) < np.float32(theta) * np.float32(D[v, u])
    reach = adj | np.eye(n, dtype=bool)
    for k in range(n):   # Floyd-Warshall transitive closure
        reach |= reach[:, k:k + 1] & reach[k:k + 1, :]
    return (reach[seeds.reshape(-1).astype(bool)].any(0)).reshape(H, W).astype(np.uint8)


def random_depth(rng, H, W):
    D = np.ones((H, W), np.float32)
    for _ in range(4):
        v0, u0 = rng.integers(0, H), rng.integers(0, W)
        D[v0:v0 + rng.integers(2, 6), u0:u0 + rng.integers(2, 6)] = rng.uniform(0.5, 3.0)
    D += rng.normal(size=(H, W)).astype(np.float32) * 0.004
    D[rng.uniform(size=(H, W)) < 0.08] = 0
    return D.astype(np.float32)


def test_floodfill_is_the_transitive_closure():
    rng = np.random.default_rng(12)
    for _ in range(12):
        H, W = rng.integers(3, 10, 2)
        D = random_depth(rng, H, W)
        seeds = ((rng.uniform(size=(H, W)) < 0.06) & (D > 0)).astype(np.uint8)
        got = O.floodfill(seeds, D, 0.007)
        assert np.array_equal(got, brute_closure(seeds, D, 0.007))


def alg1_random_order(seeds, D, theta, rng):
    """Algorithm 1 with the queue processed in random order."""
    H, W = seeds.shape
    M = np.zeros_like(seeds)
    Q = [tuple(p) for p in np.argwhere(seeds)]
    while Q:
        for p in Q:
            M[p] = 1
        rng.shuffle(Q)
        newQ = []
        for (v, u) in Q:
            for dv, du in itertools.product((-1, 0, 1), repeat=2):
                n = (v + dv, u + du)
                if (du or dv) and 0 <= n[0] < H and 0 <= n[1] < W and not M[n]:
                    if abs(np.float32(D[v, u]) - np.float32(D[n])) < np.float32(theta) * np.float32(D[v, u]):
                        newQ.append(n)
        Q = list(dict.fromkeys(newQ))
    return M


def test_floodfill_order_independent():
    rng = np.random.default_rng(13)
    for _ in range(20):
        H, W = rng.integers(5, 14, 2)
        D = random_depth(rng, H, W)
        seeds = ((rng.uniform(size=(H, W)) < 0.05) & (D > 0)).astype(np.uint8)
        ref = O.floodfill(seeds, D, 0.007)
        for _ in range(5):
            assert np.array_equal(alg1_random_order(seeds, D, 0.007, rng), ref)


def test_erosion_dilation_match_scipy():
    rng = np.random.default_rng(14)
    st = np.ones((3, 3), bool)
    for _ in range(20):
        m = (rng.uniform(size=tuple(rng.integers(1, 20, 2))) < 0.6).astype(np.uint8)
        assert np.array_equal(O.morph3x3(m, True), scipy.ndimage.binary_erosion(m, st, border_value=0))
        assert np.array_equal(O.morph3x3(m, False), scipy.ndimage.binary_dilation(m, st, border_value=0))


def test_residual_mask_marks_object_in_free_space():
    """An object appearing in front of a mapped plane lies in carved free space:
    S = tau there, r = tau^2 > gamma tau^2, so exactly its pixels are raw."""
    s, tau = 0.02, 0.06
    W, H, f = 40, 30, 30.0
    m = O.OracleMap(s, tau, 5.0, 255, 1, real_bits=32)
    bg = plane_frame(1.0, W, H, f)
    for _ in range(2):
        m.allocate(bg, np.eye(4)); m.integrate(bg, np.eye(4))
    depth = np.full((H, W), 1.0, np.float32)
    depth[10:20, 12:26] = 0.7
    fr = O.Frame(depth, np.full((H, W, 3), 50, np.uint8), f, f, (W - 1) / 2, (H - 1) / 2)
    out = m.mask(fr, np.eye(4), gamma=0.5, theta=0.007)
    obj = np.zeros((H, W), np.uint8); obj[10:20, 12:26] = 1
    assert np.array_equal(out["raw"], obj)
    np.testing.assert_allclose(out["residual"][obj == 1], np.float32(tau) ** 2, rtol=1e-6)
    assert np.all(out["residual"][obj == 0] < 1e-10)
    er = scipy.ndimage.binary_erosion(obj, np.ones((3, 3)), border_value=0)
    assert np.array_equal(out["eroded"], er)
    # flood fill grows the eroded core back over the object's flat depth
    assert np.array_equal(out["filled"], obj)
    assert np.array_equal(out["final"], scipy.ndimage.binary_dilation(obj, np.ones((3, 3))))


def test_threshold_is_strict():
    """raw = r > gamma tau^2: a residual equal to the threshold is not raw."""
    s, tau = 0.02, 0.06
    m = O.OracleMap(s, tau, 5.0, 255, 1, real_bits=32)
    bg = plane_frame(1.0)
    m.allocate(bg, np.eye(4)); m.integrate(bg, np.eye(4))
    out = m.mask(plane_frame(0.7), np.eye(4), gamma=1.0)   # r == tau^2 == gamma tau^2
    assert out["raw"].sum() == 0
    out = m.mask(plane_frame(0.7), np.eye(4), gamma=np.nextafter(np.float32(1.0), np.float32(0)))
    assert out["raw"].sum() > 0


# --- Sections III-A/III-D: block allocation ------------------------------------

def segment_cells_brute(q0, q1):
    """Cells whose closed unit box the FP64 segment q0->q1 touches, and the
    cells it touches only within 1e-4 of a box face (grazing)."""
    q0, q1 = np.asarray(q0, np.float64), np.asarray(q1, np.float64)
    lo = np.floor(np.minimum(q0, q1)).astype(int) - 1
    hi = np.floor(np.maximum(q0, q1)).astype(int) + 1
    hit, graze = set(), set()
    d = q1 - q0
    for c in itertools.product(*[range(a, b + 1) for a, b in zip(lo, hi)]):
        for eps, dest in ((-1e-4, hit), (1e-4, graze)):
            t0, t1 = 0.0, 1.0
            ok = True
            for a in range(3):
                bmin, bmax = c[a] - eps, c[a] + 1 + eps
                if d[a] == 0:
                    ok &= bmin <= q0[a] <= bmax
                else:
                    ta, tb = (bmin - q0[a]) / d[a], (bmax - q0[a]) / d[a]
                    t0, t1 = max(t0, min(ta, tb)), min(t1, max(ta, tb))
            if ok and t0 <= t1:
                dest.add(c)
    return hit, graze


def test_dda_visits_exactly_the_cells_the_segment_crosses():
    rng = np.random.default_rng(15)
    for _ in range(300):
        q0 = rng.uniform(-6, 6, 3).astype(np.float32)
        q1 = (q0 + rng.normal(size=3) * rng.choice([0.3, 2, 8])).astype(np.float32)
        cells = [tuple(c) for c in O.dda(q0, q1)]
        assert cells[0] == tuple(np.floor(q0).astype(int)) and cells[-1] == tuple(np.floor(q1).astype(int))
        steps = np.abs(np.diff(np.array(cells), axis=0)).sum(1)
        assert np.all(steps == 1)                       # 6-connected, one axis per step
        assert len(set(cells)) == len(cells)            # never revisits
        inner, outer = segment_cells_brute(q0, q1)      # inner: robustly crossed
        assert inner <= set(cells) <= outer


def test_allocation_equals_union_of_segment_cells():
    """Tiny image: F equals the union over pixels of the band (or carve) segment
    cells, with segment end points built from the FP64 pose."""
    s, tau, stride = 0.05, 0.12, 2
    W, H, f = 5, 4, 4.0
    rng = np.random.default_rng(16)
    depth = rng.uniform(0.5, 2.0, (H, W)).astype(np.float32)
    depth[1, 3] = 0
    mask = np.zeros((H, W), np.uint8); mask[2, 2] = 1
    T = O.se3_exp(np.r_[0.1, -0.2, 0.05, 0.3, 0.2, -0.1])
    fr = O.Frame(depth, np.zeros((H, W, 3), np.uint8), f, f, 2.0, 1.5)
    m = O.OracleMap(s, tau, 5.0, 255, stride, real_bits=32)
    F = {tuple(k) for k in m.allocate(fr, T, mask)}
    B = 8 * float(np.float32(s))
    inner_all, outer_all = set(), set()
    for v, u in itertools.product(range(H), range(W)):
        D = float(depth[v, u])
        if D <= 0 or mask[v, u]:
            continue
        carve = (u % stride == 0) and (v % stride == 0)
        zn, zf = (0.0 if carve else max(D - tau, 0.0)), D + tau
        ray = np.array([(u - 2.0) / f, (v - 1.5) / f, 1.0])
        p0, p1 = T[:3, :3] @ (ray * zn) + T[:3, 3], T[:3, :3] @ (ray * zf) + T[:3, 3]
        inner, outer = segment_cells_brute(p0 / B, p1 / B)
        inner_all |= inner
        outer_all |= outer
    assert inner_all <= F <= outer_all
    assert m.num_blocks == len(F)


# ---------------------------------------------------------------- mesh (marching tetrahedra)

def sphere_mesh(centre, r, s=0.01, tau=0.05, real_bits=64, hole=None):
    """Oracle mesh of an exact sphere SDF (clamped to +-tau) sampled at the
    voxel centres of every block near the sphere; hole: voxel index whose
    weight is zeroed."""
    ang = np.linspace(0, 2 * np.pi, 90)
    pol = np.linspace(0, np.pi, 45)
    pts = centre + r * np.array([[np.cos(a) * np.sin(b), np.sin(a) * np.sin(b), np.cos(b)] for a in ang for b in pol])
    keys = A.blocks_near(pts, s, 1)
    k, sdf, w, rgb = A.fill_map(keys, s, lambda x: np.clip(np.linalg.norm(x - centre, axis=-1) - r, -tau, tau))
    if hole is not None:
        v = np.asarray(hole)
        b, l = v // 8, v % 8
        i = np.nonzero((k == b).all(1))[0][0]
        w[i, l[0] + 8 * l[1] + 64 * l[2]] = 0.0
    om = O.OracleMap(s, tau, 5.0, 255, 4, real_bits=real_bits)
    om.import_(k, sdf, w, rgb)
    return om.mesh()


def test_mesh_of_sphere_matches_closed_form():
    c, r = np.array([0.013, -0.007, 0.021]), 0.2
    T = sphere_mesh(c, r)
    V = T.reshape(-1, 3)
    # vertices: crossings of chords of length <= sqrt(3) s, so within (sqrt(3) s)^2 / (8 r) of the sphere
    assert np.abs(np.linalg.norm(V - c, axis=1) - r).max() <= 3 * 0.01 ** 2 / (8 * r) * 1.01
    area = 0.5 * np.linalg.norm(np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0]), axis=1).sum()
    vol = np.einsum("ij,ij->i", T[:, 0] - c, np.cross(T[:, 1] - c, T[:, 2] - c)).sum() / 6.0
    assert abs(area / (4 * np.pi * r * r) - 1) < 2e-3
    assert abs(vol / (4.0 / 3.0 * np.pi * r ** 3) - 1) < 2e-3   # positive: normals face outward


def test_mesh_is_closed_and_consistently_oriented():
    T = sphere_mesh(np.array([0.004, 0.011, -0.002]), 0.12)
    V, idx = np.unique(T.reshape(-1, 3), axis=0, return_inverse=True)
    F = idx.reshape(-1, 3)
    assert (F[:, 0] != F[:, 1]).all() and (F[:, 1] != F[:, 2]).all() and (F[:, 0] != F[:, 2]).all()
    directed = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]])
    d_set = set(map(tuple, directed))
    assert len(d_set) == len(directed)                         # each directed edge once
    assert all((b, a) in d_set for a, b in d_set)              # and its reverse once: closed, oriented
    E = len(directed) // 2
    assert len(V) - E + len(F) == 2                            # Euler characteristic of a sphere


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_mesh_of_plane_lies_on_the_plane(seed):
    rng = np.random.default_rng(seed)
    n = rng.normal(size=3)
    n /= np.linalg.norm(n)
    d0 = rng.uniform(-0.02, 0.02)
    s, tau = 0.01, 0.06
    keys = np.array([[x, y, z] for x in range(-1, 1) for y in range(-1, 1) for z in range(-1, 1)], np.int32)
    k, sdf, w, rgb = A.fill_map(keys, s, lambda x: np.clip(x @ n - d0, -tau, tau))
    om = O.OracleMap(s, tau, 5.0, 255, 4, real_bits=64)
    om.import_(k, sdf, w, rgb)
    T = om.mesh()
    assert len(T) > 100
    assert np.abs(T.reshape(-1, 3) @ n - d0).max() < 1e-12      # a linear field is interpolated exactly
    nrm = np.cross(T[:, 1] - T[:, 0], T[:, 2] - T[:, 0])
    big = np.linalg.norm(nrm, axis=1) > 1e-10
    assert (nrm[big] @ n > 0).all()                            # facing the positive side


def test_mesh_skips_cubes_with_an_unobserved_corner():
    c, r = np.array([0.0, 0.0, 0.0]), 0.1
    full = sphere_mesh(c, r)
    v = np.array([10, 0, 0])                                   # a voxel on the sphere (x = 0.1 m)
    holed = sphere_mesh(c, r, hole=v)
    lo = v * 0.01 - 0.01 - 1e-9
    hi = v * 0.01 + 0.01 + 1e-9
    inside = lambda T: ((T >= lo) & (T <= hi)).all(axis=2).all(axis=1)
    # the 8 cubes around the voxel lose all their triangles; nothing else changes
    keep = ~inside(full)
    assert inside(full).sum() > 0 and inside(holed).sum() == 0
    a = np.sort(full[keep].reshape(len(full[keep]), -1), axis=0)
    b = np.sort(holed.reshape(len(holed), -1), axis=0)
    assert a.shape == b.shape and np.array_equal(a, b)


def test_mesh_fp32_mirror_close_to_fp64():
    c, r = np.array([0.013, -0.007, 0.021]), 0.15
    T64 = sphere_mesh(c, r)
    T32 = sphere_mesh(c, r, real_bits=32)
    assert T64.shape == T32.shape                   # same cubes, same cases, same emission order
    assert np.abs(T64 - T32).max() < 1e-6


# ---------------------------------------------------------------- virtual depth (ray cast)

def plane_map(n, c, s=0.01, tau=0.05, extent=((-0.9, 0.9), (-0.7, 0.7), (0.8, 2.2)), real_bits=64):
    """Oracle map of the plane n.x = c (SDF positive on the camera side,
    n pointing away from the camera) over the blocks of a box."""
    B = 8 * s
    rng_ = [np.arange(int(np.floor(lo / B)), int(np.floor(hi / B)) + 1) for lo, hi in extent]
    keys = np.array([[x, y, z] for x in rng_[0] for y in rng_[1] for z in rng_[2]], np.int32)
    k, sdf, w, rgb = A.fill_map(keys, s, lambda x: np.clip(c - x @ n, -tau, tau))
    om = O.OracleMap(s, tau, 5.0, 255, 4, real_bits=real_bits)
    om.import_(k, sdf.astype(np.float32).astype(np.float64), w, rgb)
    return om


def pinhole_frame(W=40, H=30, f=30.0, depth=None):
    d = np.zeros((H, W), np.float32) if depth is None else depth.astype(np.float32)
    return O.Frame(d, np.zeros((H, W, 3), np.uint8), f, f, (W - 1) / 2.0, (H - 1) / 2.0)


@pytest.mark.parametrize("tilt", [0.0, 0.25, 0.5])
def test_raycast_of_plane_matches_closed_form(tilt):
    n = np.array([0.0, np.sin(tilt), np.cos(tilt)])
    c = 1.3
    om = plane_map(n, c)
    fr = pinhole_frame()
    z = om.raycast(fr, np.eye(4), z_near=0.3, z_far=5.0, only_invalid=False)
    v, u = np.mgrid[0:fr.H, 0:fr.W]
    d = np.stack([(u - fr.s.cx) / fr.s.fx, (v - fr.s.cy) / fr.s.fy, np.ones_like(u, float)], -1)
    exact = c / (d @ n)                              # camera depth of the plane along each ray
    P = exact[..., None] * d                         # where they meet it
    inside = ((np.abs(P[..., 0]) < 0.85) & (np.abs(P[..., 1]) < 0.65)
              & (exact > 0.85) & (exact < 2.1))       # inside the mapped box, two voxels from its faces
    assert inside.sum() > 500
    # the plane's TSDF is linear, so the trilinear samples and the crossing are exact up to rounding
    assert np.abs(z[inside] - exact[inside]).max() < 2e-6


def test_raycast_of_sphere_matches_ray_intersection():
    s, tau = 0.01, 0.05
    c, r = np.array([0.05, -0.03, 1.2]), 0.3
    ang = np.linspace(0, 2 * np.pi, 90)
    pol = np.linspace(0, np.pi, 45)
    pts = c + r * np.array([[np.cos(a) * np.sin(b), np.sin(a) * np.sin(b), np.cos(b)] for a in ang for b in pol])
    keys = A.blocks_near(pts, s, 1)
    k, sdf, w, rgb = A.fill_map(keys, s, lambda x: np.clip(np.linalg.norm(x - c, axis=-1) - r, -tau, tau))
    om = O.OracleMap(s, tau, 5.0, 255, 4, real_bits=64)
    om.import_(k, sdf, w, rgb)
    fr = pinhole_frame(W=48, H=36, f=40.0)
    z = om.raycast(fr, np.eye(4), only_invalid=False)
    v, u = np.mgrid[0:fr.H, 0:fr.W]
    d = np.stack([(u - fr.s.cx) / fr.s.fx, (v - fr.s.cy) / fr.s.fy, np.ones_like(u, float)], -1)
    # first intersection of z d with the sphere: |z d - c|^2 = r^2
    a = (d * d).sum(-1)
    b = (d @ c)
    disc = b * b - a * (c @ c - r * r)
    exact = (b - np.sqrt(np.maximum(disc, 0))) / a
    nrm = (exact[..., None] * d - c) / r
    cosi = np.abs((nrm * d).sum(-1)) / np.sqrt(a)
    hitp = (disc > 0) & (cosi > 0.5)                 # rays meeting the sphere at incidence below 60 degrees
    assert hitp.sum() > 100
    assert np.abs(z[hitp] - exact[hitp]).max() < 1e-3
    assert (z[~(disc > 0)] == 0).all()               # rays that miss report no crossing


def test_raycast_fills_only_zero_depth():
    n, c = np.array([0.0, 0.0, 1.0]), 1.3
    om = plane_map(n, c)
    rng = np.random.default_rng(3)
    depth = rng.uniform(0.5, 4.0, (30, 40)).astype(np.float32)
    holes = rng.uniform(size=depth.shape) < 0.3
    depth[holes] = 0.0
    depth[0, :] = 0.0                                # top row: rays through the mapped box
    fr = pinhole_frame(depth=depth)
    out = om.raycast(fr, np.eye(4), far_value=4.5, only_invalid=True)
    assert np.array_equal(out[~holes & (np.arange(30)[:, None] > 0)], depth[~holes & (np.arange(30)[:, None] > 0)])
    filled = out[depth == 0]
    assert np.all((np.abs(filled - 1.3) < 2e-6) | (filled == np.float32(4.5)))
    assert (np.abs(filled - 1.3) < 2e-6).mean() > 0.9
    # a camera looking away from the model gets the far value everywhere it had zeros
    away = np.diag([1.0, 1.0, -1.0, 1.0])
    away[0, 0] = -1.0
    out2 = om.raycast(fr, away, far_value=4.5, only_invalid=True)
    assert np.all(out2[depth == 0] == np.float32(4.5))
