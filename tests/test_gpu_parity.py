"""GPU (HIP, gfx950) vs CPU oracle parity on seeded synthetic inputs.

Bars: allocated block sets and dynamic masks bit-exact; voxel values
bit-exact against the FP32 mirror (same FP32 decision and value order) and
within 1e-5 m of the FP64 reference; poses within 1e-4 m / 1e-5 rad of the
FP64 reference."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from gpu_helpers import (dev_pose, gpu_export_sorted, gpu_frame, gpu_keyset, map_params, need_gpu, orc_frame,
                         oracle_maps, pose_error, sort_keys)

pytestmark = pytest.mark.gpu


def track_stats(stats):
    """(iterations applied, flags) of a device rf_track_stats buffer."""
    u = stats.cpu().numpy().view(np.uint32)
    return int(u[4]), int(u[5])


@pytest.fixture(scope="module")
def rf():
    return need_gpu()


@pytest.fixture(scope="module")
def room():
    return synth.parity_room()


@pytest.fixture(scope="module")
def dyn_small():
    return synth.dynamic_room(n_frames=24, width=160, height=120, n_clusters=2, movers="in_view")


def integrate_teacher_forced(rf, seq, frames, storage="fp32", orc_storage=0, masks=None, max_blocks=None):
    """Integrates the given frames at ground-truth poses on the GPU and both
    oracle maps; returns (gpu map, fp64 oracle, fp32 mirror)."""
    m = rf.Map(map_params(rf, seq, storage, max_blocks=max_blocks))
    o64, o32 = oracle_maps(seq, orc_storage)
    for i, k in enumerate(frames):
        mk = None if masks is None else masks[i]
        g = gpu_frame(rf, seq, k)
        P = dev_pose(seq.poses[k])
        mt = None if mk is None else torch.from_numpy(mk).cuda()
        m.allocate(g, P, mt)
        m.integrate(g, P, mt)
        fr = orc_frame(seq, k)
        for o in (o64, o32):
            o.allocate(fr, seq.poses[k], mk)
            o.integrate(fr, seq.poses[k], mk)
    torch.cuda.synchronize()
    return m, o64, o32


def assert_maps_match(m, o64, o32, sdf_tol=1e-5):
    gk, gs, gw, gc = gpu_export_sorted(m)
    k32, s32, w32, c32 = o32.export()
    k64, s64, w64, c64 = o64.export()
    assert np.array_equal(gk, k32) and np.array_equal(gk, k64)
    np.testing.assert_array_equal(gs, s32.astype(np.float32))      # bit-exact vs FP32 mirror
    np.testing.assert_array_equal(gw, w32.astype(np.float32))
    np.testing.assert_array_equal(gc, c32)
    assert np.max(np.abs(gs.astype(np.float64) - s64)) <= sdf_tol   # vs FP64 reference
    np.testing.assert_array_equal(gw, w64.astype(np.float32))
    np.testing.assert_array_equal(gc, c64)


# ---------------------------------------------------------------- allocation

def test_allocation_block_set_bit_exact(rf, room):
    m = rf.Map(map_params(rf, room))
    o = O.OracleMap(room.voxel_size, room.truncation, room.depth_max, 255, room.carve_stride, real_bits=32)
    rng = np.random.default_rng(0)
    for k in range(3):
        mask = (rng.uniform(size=(room.height, room.width)) < 0.1).astype(np.uint8) if k == 2 else None
        g = gpu_frame(rf, room, k)
        m.allocate(g, dev_pose(room.poses[k]), None if mask is None else torch.from_numpy(mask).cuda())
        F_gpu = gpu_keyset(m.frame_blocks())
        F_orc = o.allocate(orc_frame(room, k), room.poses[k], mask)
        assert np.array_equal(F_gpu, F_orc), k
    flags, nb = m.status()
    assert flags == 0 and nb == o.num_blocks
    gk = gpu_export_sorted(m)[0]
    assert np.array_equal(gk, o.export()[0])


# ---------------------------------------------------------------- integration

def test_integration_matches_oracle(rf, room):
    m, o64, o32 = integrate_teacher_forced(rf, room, range(3))
    assert_maps_match(m, o64, o32)
    # one more frame: the update counts (band, free) agree with the mirror's
    g = gpu_frame(rf, room, 3)
    P = dev_pose(room.poses[3])
    m.allocate(g, P)
    m.integrate(g, P)
    o64.allocate(orc_frame(room, 3), room.poses[3])
    o64.integrate(orc_frame(room, 3), room.poses[3])
    o32.allocate(orc_frame(room, 3), room.poses[3])
    cnt = o32.integrate(orc_frame(room, 3), room.poses[3])
    torch.cuda.synchronize()
    assert m.stats_counts() == (int(cnt[0]), int(cnt[1]))
    assert_maps_match(m, o64, o32)


def test_integration_masked_pixels_untouched(rf, room):
    rng = np.random.default_rng(1)
    mask = np.zeros((room.height, room.width), np.uint8)
    mask[30:80, 40:100] = 1
    masks = [None, mask, (rng.uniform(size=mask.shape) < 0.3).astype(np.uint8)]
    m, o64, o32 = integrate_teacher_forced(rf, room, range(3), masks=masks)
    assert_maps_match(m, o64, o32)


@pytest.mark.parametrize("storage,orc_storage", [("fp32", 0), ("fp16", 1)])
def test_far_measurements_carve_up_to_clipping_plane(rf, room, storage, orc_storage):
    """Clipping plane at 1.2 m in the 2 m room: most measurements lie beyond
    it; they add no band but carve free space in front of the plane along
    their carve rays (Sec. III-D).  Block sets and voxels bit-exact against
    the mirror, and the far pixels really carve (more free updates than with
    those pixels removed from the frame)."""
    import dataclasses
    near = dataclasses.replace(room, depth_max=1.2)
    d0 = synth.depth_metres(near, 0)
    assert (d0 > 1.2).mean() > 0.5
    m, o64, o32 = integrate_teacher_forced(rf, near, range(3), storage=storage, orc_storage=orc_storage)
    gk, gs, gw, gc = gpu_export_sorted(m)
    k32, s32, w32, c32 = o32.export()
    assert np.array_equal(gk, k32)
    np.testing.assert_array_equal(gs, s32.astype(np.float32))
    np.testing.assert_array_equal(gw, w32.astype(np.float32))
    np.testing.assert_array_equal(gc, c32)
    # the same frame with its far pixels cleared carves less
    cut = dataclasses.replace(near, depth=near.depth.copy())
    for k in range(near.n):
        cut.depth[k][synth.depth_metres(near, k) > 1.2] = 0
    m2 = rf.Map(map_params(rf, cut, storage))
    for k in range(3):
        g = gpu_frame(rf, cut, k)
        P = dev_pose(cut.poses[k])
        m2.allocate(g, P)
        m2.integrate(g, P)
    torch.cuda.synchronize()
    assert m2.status()[1] < m.status()[1]


def test_integration_fp16_storage_matches_mirror(rf, room):
    m, o64, o16 = integrate_teacher_forced(rf, room, range(4), storage="fp16", orc_storage=1)
    gk, gs, gw, gc = gpu_export_sorted(m)
    k16, s16, w16, c16 = o16.export()
    assert np.array_equal(gk, k16)
    np.testing.assert_array_equal(gs, s16.astype(np.float32))
    np.testing.assert_array_equal(gw, w16.astype(np.float32))
    np.testing.assert_array_equal(gc, c16)
    k64, s64, w64, _ = o64.export()
    assert np.array_equal(gk, k64)
    obs = w64 > 0
    err = np.abs(gs.astype(np.float64) - s64)[obs]
    # each FP16 store of sdf/tau rounds by at most 2^-12 tau (half an ulp in
    # [0.5, 1)); the running average carries earlier errors with factor
    # W/(W+1), so after n updates the error is at most n 2^-12 tau
    assert err.max() <= 4 * room.truncation * 2.0 ** -12


# ---------------------------------------------------------------- tracking

def test_normal_equations_match_oracle(rf, room):
    m, o64, o32 = integrate_teacher_forced(rf, room, range(2))
    rng = np.random.default_rng(2)
    g = gpu_frame(rf, room, 2)
    fr = orc_frame(room, 2)
    for level in (0, 1):
        T = O.pose_left_update(np.r_[rng.normal(size=3) * 0.005, rng.normal(size=3) * 0.003], room.poses[1])
        ne = m.normal_equations(g, dev_pose(T), level, 0.025).cpu().numpy()
        ne32 = o32.normal_equations(fr, T, level, 0.025)
        ne64 = o64.normal_equations(fr, T, level, 0.025)
        assert ne[28] == ne32[28] and ne[28] > 1000                    # identical FP32 decisions
        scale = np.abs(ne32[:28]).max()
        assert np.max(np.abs(ne[:28] - ne32[:28])) <= 1e-12 * scale * ne[28]
        assert abs(ne[28] - ne64[28]) <= 0.002 * ne64[28]
        np.testing.assert_allclose(ne[:21], ne64[:21], rtol=2e-3, atol=2e-3 * np.abs(ne64[:21]).max())


def test_track_pose_matches_fp64_oracle(rf, room):
    m, o64, o32 = integrate_teacher_forced(rf, room, range(1))
    tp = rf.TrackParams(room.levels, room.iters)
    for k in (1, 2):
        P = dev_pose(room.poses[0])
        stats = torch.zeros(16, dtype=torch.float64, device="cuda")
        m.track(gpu_frame(rf, room, k), P, tp, None, stats)
        T_ref, flags, st = o64.track(orc_frame(room, k), room.poses[0], room.levels, room.iters)
        T_gpu = P.cpu().numpy()
        dt, dr = pose_error(T_gpu, T_ref)
        assert flags == 0
        assert dt <= 1e-4 and dr <= 1e-5, (k, dt, dr)
        iters, fl = track_stats(stats)
        assert iters == room.levels * room.iters and fl == 0


@pytest.mark.parametrize("lam0", [1e-4, 0.0])
def test_track_lm_pose_matches_fp64_oracle(rf, room, lam0):
    """Levenberg-Marquardt schedule (accept / reject on the mean cost): the GPU
    decisions are taken on fixed-point totals, the oracle's on FP64 sums, so a
    near-tie may be decided differently; the poses still agree to the bar."""
    m, o64, o32 = integrate_teacher_forced(rf, room, range(2))
    tp = rf.TrackParams(room.levels, room.iters, lm_lambda=lam0, adaptive=True)
    for k in (2, 3):
        T0 = room.poses[1]
        P = dev_pose(T0)
        stats = torch.zeros(16, dtype=torch.float64, device="cuda")
        m.track(gpu_frame(rf, room, k), P, tp, None, stats)
        T_ref, flags, st, trace = o64.track_lm(orc_frame(room, k), T0, room.levels, room.iters, lambda0=lam0)
        assert flags == 0
        dt, dr = pose_error(P.cpu().numpy(), T_ref)
        assert dt <= 1e-4 and dr <= 1e-5, (k, dt, dr)
        iters, fl = track_stats(stats)
        assert fl == 0 and 0 < iters <= room.levels * (room.iters - 1)
        assert abs(iters - int(st[2])) <= 2
        gt_t, _ = pose_error(P.cpu().numpy(), room.poses[k])
        assert gt_t < 5e-3


def test_free_running_parity_room_poses(rf, room):
    """10 frames free-running: GPU pipeline vs FP64 oracle pipeline."""
    tp = rf.TrackParams(room.levels, room.iters)
    pipe = rf.Pipeline(map_params(rf, room), tp, rf.MaskParams(), room.poses[0], dynamic=True)
    o64, o32 = oracle_maps(room)
    T = room.poses[0]
    for k in range(room.n):
        pipe.process(gpu_frame(rf, room, k))
        T, _ = O.process_frame(o64, orc_frame(room, k), T, k, room.levels, room.iters, mask_map=o32)
        dt, dr = pose_error(pipe.pose.cpu().numpy(), T)
        assert dt <= 1e-4 and dr <= 1e-5, (k, dt, dr)
    assert pipe.map.status()[0] == 0


# ---------------------------------------------------------------- dynamic mask

@pytest.mark.parametrize("k", [12, 20])
def test_dynamic_mask_stages_bit_exact(rf, dyn_small, k):
    seq = dyn_small
    masks = [(seq.labels[j] > 0).astype(np.uint8) for j in range(0, k, 3)]
    m, o64, o32 = integrate_teacher_forced(rf, seq, range(0, k, 3), masks=masks)
    g = gpu_frame(rf, seq, k)
    res = torch.empty((seq.height, seq.width), dtype=torch.float32, device="cuda")
    out = m.dynamic_mask(g, dev_pose(seq.poses[k]), rf.MaskParams(0.5, 0.007), residual=res, stages=True)
    ref = o32.mask(orc_frame(seq, k), seq.poses[k], 0.5, 0.007)
    for key in ("raw", "eroded", "filled", "final"):
        assert np.array_equal(out[key].cpu().numpy(), ref[key]), key
    np.testing.assert_array_equal(res.cpu().numpy(), ref["residual"])
    assert ref["raw"].sum() > 20 and ref["final"].sum() > ref["eroded"].sum()


def test_flood_fill_across_the_whole_frame(rf):
    """A map of a fronto-parallel wall at 2 m; the frame sees a plane slanted
    from 1.90 m (top left) to 2.50 m (bottom right): only a corner lies in
    front of the wall by more than the residual threshold, and the flood fill
    grows from its eroded seeds over the whole plane (neighbouring depths
    differ by ~1 mm, far below theta D), about 35 tile steps, so most of the
    growth is left to the one-workgroup drain after the parallel passes.  All
    mask stages are bit-exact against the FP32 mirror."""
    W, H = 640, 480
    intr = (525.0, 525.0, 319.5, 239.5)
    rgb = np.full((H, W, 3), 128, np.uint8)
    wall = np.full((H, W), 2.0, np.float32)
    uu, vv = np.meshgrid(np.arange(W, dtype=np.float64), np.arange(H, dtype=np.float64))
    slant = (1.90 + 0.6 * (uu / (W - 1) + vv / (H - 1)) / 2.0).astype(np.float32)
    T = np.eye(4)
    params = rf.MapParams(0.01, 0.03, 5.0, 1 << 16, 1 << 14, 255, 2, "fp32", W * H)
    m = rf.Map(params)
    g0 = rf.Frame.from_numpy(wall, rgb, *intr)
    P = dev_pose(T)
    m.allocate(g0, P)
    m.integrate(g0, P)
    o32 = O.OracleMap(0.01, 0.03, 5.0, 255, 2, real_bits=32)
    f0 = O.Frame(wall, rgb, *intr)
    o32.allocate(f0, T)
    o32.integrate(f0, T)
    g1 = rf.Frame.from_numpy(slant, rgb, *intr)
    out = m.dynamic_mask(g1, P, rf.MaskParams(0.5, 0.007), stages=True)
    ref = o32.mask(O.Frame(slant, rgb, *intr), T, 0.5, 0.007)
    for key in ("raw", "eroded", "filled", "final"):
        assert np.array_equal(out[key].cpu().numpy(), ref[key]), key
    assert 0 < ref["eroded"].sum() < 0.05 * W * H and ref["filled"].sum() > 0.9 * W * H
    assert m.status()[0] == 0


# ---------------------------------------------------------------- surface / checkpoint

def test_extract_surface_matches_mirror(rf, room):
    m, o64, o32 = integrate_teacher_forced(rf, room, range(3))
    pts = m.surface().cpu().numpy().astype(np.float64)
    ref = o32.surface()
    assert len(pts) == len(ref) and len(ref) > 1000
    key = lambda p: np.lexsort((p[:, 6], p[:, 2], p[:, 1], p[:, 0]))
    np.testing.assert_array_equal(pts[key(pts)], ref[key(ref)])


def test_export_import_roundtrip(rf, room):
    m, _, _ = integrate_teacher_forced(rf, room, range(2))
    keys, sdf, w, rgb = m.export()
    m2 = rf.Map(map_params(rf, room))
    m2.import_(keys, sdf, w, rgb)
    a = gpu_export_sorted(m)
    b = gpu_export_sorted(m2)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


# ---------------------------------------------------------------- edge cases

def test_empty_frame(rf, room):
    m = rf.Map(map_params(rf, room))
    z = np.zeros((room.height, room.width), np.float32)
    g = rf.Frame.from_numpy(z, room.rgb[0], *room.intrinsics)
    P = dev_pose(room.poses[0])
    m.allocate(g, P)
    m.integrate(g, P)
    assert m.status() == (0, 0)
    stats = torch.zeros(16, dtype=torch.float64, device="cuda")
    m.track(g, P, rf.TrackParams(2, 3), None, stats)
    assert np.array_equal(P.cpu().numpy(), room.poses[0])
    iters, fl = track_stats(stats)
    assert iters == 0 and fl & rf.RF_FLAG_TRACK_FEW_PIXELS
    mk = m.dynamic_mask(g, P, rf.MaskParams())
    assert int(mk.sum()) == 0


def test_ragged_image_sizes(rf):
    seq = synth.dynamic_room(n_frames=8, width=77, height=53, n_clusters=1, movers="in_view")
    masks = [None, None, None]
    m, o64, o32 = integrate_teacher_forced(rf, seq, range(0, 6, 2), masks=masks)
    assert_maps_match(m, o64, o32)
    g = gpu_frame(rf, seq, 7)
    out = m.dynamic_mask(g, dev_pose(seq.poses[7]), rf.MaskParams(), stages=True)
    ref = o32.mask(orc_frame(seq, 7), seq.poses[7], 0.5, 0.007)
    for key in ("raw", "eroded", "filled", "final"):
        assert np.array_equal(out[key].cpu().numpy(), ref[key]), key


def test_pool_and_hash_full_flags(rf, room):
    m = rf.Map(map_params(rf, room, max_blocks=50))
    g = gpu_frame(rf, room, 0)
    P = dev_pose(room.poses[0])
    m.allocate(g, P)
    m.integrate(g, P)
    flags, nb = m.status()
    assert flags & rf.RF_FLAG_POOL_FULL and nb == 50
    m = rf.Map(map_params(rf, room, num_buckets=64))
    m.allocate(g, P)
    m.integrate(g, P)
    flags, nb = m.status()
    assert flags & rf.RF_FLAG_HASH_FULL and nb == 64


def test_bad_arguments_raise(rf, room):
    with pytest.raises(rf.RefusionError):
        rf.Map(rf.MapParams(0.01, 0.03, num_buckets=1000))
    m = rf.Map(map_params(rf, room))
    g = gpu_frame(rf, room, 0)
    with pytest.raises(rf.RefusionError):
        m.track(g, dev_pose(room.poses[0]), rf.TrackParams(levels=9))
    big = rf.Frame.from_numpy(np.zeros((200, 200), np.float32), np.zeros((200, 200, 3), np.uint8), 100, 100, 99, 99)
    with pytest.raises(rf.RefusionError):
        m.dynamic_mask(big, dev_pose(room.poses[0]), rf.MaskParams())


# ---------------------------------------------------------------- full size (640x480)

@pytest.fixture(scope="module")
def static_seq():
    return synth.static_room(n_frames=4)


def test_full_size_static_room_teacher_forced(rf, static_seq):
    seq = static_seq
    m = rf.Map(map_params(rf, seq, max_blocks=1 << 17))
    o32 = O.OracleMap(seq.voxel_size, seq.truncation, seq.depth_max, 255, seq.carve_stride, real_bits=32)
    for k in range(2):
        g = gpu_frame(rf, seq, k)
        P = dev_pose(seq.poses[k])
        m.allocate(g, P)
        F_gpu = gpu_keyset(m.frame_blocks())
        F_orc = o32.allocate(orc_frame(seq, k), seq.poses[k])
        assert np.array_equal(F_gpu, F_orc), k
        m.integrate(g, P)
        o32.integrate(orc_frame(seq, k), seq.poses[k])
    gk, gs, gw, gc = gpu_export_sorted(m)
    k32, s32, w32, c32 = o32.export()
    assert np.array_equal(gk, k32)
    np.testing.assert_array_equal(gs, s32.astype(np.float32))
    np.testing.assert_array_equal(gw, w32.astype(np.float32))
    np.testing.assert_array_equal(gc, c32)
    # the registration step at full size: identical FP32 decisions, sums to FP64 rounding
    g = gpu_frame(rf, seq, 2)
    ne = m.normal_equations(g, dev_pose(seq.poses[1]), 0, 0.025).cpu().numpy()
    ne32 = o32.normal_equations(orc_frame(seq, 2), seq.poses[1], 0, 0.025)
    assert ne[28] == ne32[28] and ne[28] > 50000
    assert np.max(np.abs(ne[:28] - ne32[:28])) <= 1e-12 * np.abs(ne32[:28]).max() * ne[28]
    out = m.dynamic_mask(g, dev_pose(seq.poses[2]), rf.MaskParams(), stages=True)
    ref = o32.mask(orc_frame(seq, 2), seq.poses[2], 0.5, 0.007)
    for key in ("raw", "eroded", "filled", "final"):
        assert np.array_equal(out[key].cpu().numpy(), ref[key]), key


@pytest.fixture(scope="module")
def dyn_full():
    """640x480 dynamic room, movers in view from frame 0 (13 frames)."""
    return synth.dynamic_room(n_frames=13, movers="in_view")


@pytest.fixture(scope="module")
def dyn_full_maps(rf, dyn_full):
    """The dynamic room fused at ground-truth poses with ground-truth masks
    (frames 0, 3, 6, 9), on the GPU and both oracle maps."""
    seq = dyn_full
    ks = list(range(0, 12, 3))
    masks = [(seq.labels[k] > 0).astype(np.uint8) for k in ks]
    m = rf.Map(map_params(rf, seq, max_blocks=1 << 17))
    o64, o32 = oracle_maps(seq)
    for k, mk in zip(ks, masks):
        g = gpu_frame(rf, seq, k)
        P = dev_pose(seq.poses[k])
        mt = torch.from_numpy(mk).cuda()
        m.allocate(g, P, mt)
        m.integrate(g, P, mt)
        for o in (o64, o32):
            o.allocate(orc_frame(seq, k), seq.poses[k], mk)
            o.integrate(orc_frame(seq, k), seq.poses[k], mk)
    torch.cuda.synchronize()
    return m, o64, o32


def test_full_size_dynamic_room_mask_stages(rf, dyn_full, dyn_full_maps):
    """640x480 frame with movers in view: residual, raw, eroded, flood-filled
    and final masks bit-exact against the FP32 mirror, on non-trivial content
    (the fill grows the eroded seeds across many 32x32 tiles)."""
    seq = dyn_full
    m, _, o32 = dyn_full_maps
    assert_maps_match(m, dyn_full_maps[1], o32)
    k = 12
    g = gpu_frame(rf, seq, k)
    res = torch.empty((seq.height, seq.width), dtype=torch.float32, device="cuda")
    out = m.dynamic_mask(g, dev_pose(seq.poses[k]), rf.MaskParams(0.5, 0.007), residual=res, stages=True)
    ref = o32.mask(orc_frame(seq, k), seq.poses[k], 0.5, 0.007)
    np.testing.assert_array_equal(res.cpu().numpy(), ref["residual"])
    for key in ("raw", "eroded", "filled", "final"):
        assert np.array_equal(out[key].cpu().numpy(), ref[key]), key
    assert ref["eroded"].sum() > 1000 and ref["filled"].sum() > 2 * ref["eroded"].sum()
    filled_tiles = {(v // 32, u // 32) for v, u in zip(*np.nonzero(ref["filled"]))}
    assert len(filled_tiles) > 30


def test_full_size_dynamic_room_three_level_poses(rf, dyn_full, dyn_full_maps):
    """Both registration passes of a 640x480 dynamic frame, 3 levels x 10
    iterations, against the FP64 oracle from the same start: pass 1 without a
    mask, pass 2 with the mask the FP32 mirror computes at the FP64 pass-1
    pose; within 1e-4 m / 1e-5 rad."""
    seq = dyn_full
    m, o64, o32 = dyn_full_maps
    k = 12
    tp = rf.TrackParams(seq.levels, seq.iters)
    g, fr = gpu_frame(rf, seq, k), orc_frame(seq, k)
    T0 = seq.poses[k - 3]
    P = dev_pose(T0)
    m.track(g, P, tp)
    T1, fl, _ = o64.track(fr, T0, seq.levels, seq.iters)
    assert fl == 0
    dt, dr = pose_error(P.cpu().numpy(), T1)
    assert dt <= 1e-4 and dr <= 1e-5, (dt, dr)
    M = o32.mask(fr, T1, 0.5, 0.007)["final"]
    assert M.sum() > 10000
    P = dev_pose(T1)
    m.track(g, P, tp, torch.from_numpy(M).cuda())
    T2, fl, _ = o64.track(fr, T1, seq.levels, seq.iters, mask=M)
    assert fl == 0
    dt, dr = pose_error(P.cpu().numpy(), T2)
    assert dt <= 1e-4 and dr <= 1e-5, (dt, dr)


def test_full_size_static_room_three_level_pose(rf, static_seq):
    """640x480 static room, registration of frame 3 from frame 2's pose with
    3 levels x 10 iterations on a map of frames 0-2: within 1e-4 m / 1e-5 rad
    of the FP64 oracle."""
    seq = static_seq
    m = rf.Map(map_params(rf, seq, max_blocks=1 << 17))
    o64 = O.OracleMap(seq.voxel_size, seq.truncation, seq.depth_max, 255, seq.carve_stride, real_bits=64)
    for k in range(3):
        g = gpu_frame(rf, seq, k)
        P = dev_pose(seq.poses[k])
        m.allocate(g, P)
        m.integrate(g, P)
        o64.allocate(orc_frame(seq, k), seq.poses[k])
        o64.integrate(orc_frame(seq, k), seq.poses[k])
    P = dev_pose(seq.poses[2])
    m.track(gpu_frame(rf, seq, 3), P, rf.TrackParams(seq.levels, seq.iters))
    T, fl, _ = o64.track(orc_frame(seq, 3), seq.poses[2], seq.levels, seq.iters)
    assert fl == 0
    dt, dr = pose_error(P.cpu().numpy(), T)
    assert dt <= 1e-4 and dr <= 1e-5, (dt, dr)
    assert pose_error(T, seq.poses[3])[0] < 2e-2


@pytest.mark.parametrize("storage,orc_storage", [("fp32", 0), ("fp16", 1)])
def test_full_size_large_rooms_integration(rf, storage, orc_storage):
    """The 0.5 cm-voxel large rooms, two 640x480 frames fused at ground-truth
    poses (~65 k blocks per frame, measurements beyond the clipping plane
    carving in front of it): voxels bit-exact against the FP32 (FP16) mirror
    and the FP32 sdf within 1e-5 m of FP64."""
    seq = synth.large_rooms(n_frames=2)
    m, o64, om = integrate_teacher_forced(rf, seq, range(2), storage=storage, orc_storage=orc_storage,
                                          max_blocks=1 << 18)
    gk, gs, gw, gc = gpu_export_sorted(m)
    km, sm, wm, cm = om.export()
    assert np.array_equal(gk, km) and len(gk) > 50000
    np.testing.assert_array_equal(gs, sm.astype(np.float32))
    np.testing.assert_array_equal(gw, wm.astype(np.float32))
    np.testing.assert_array_equal(gc, cm)
    k64, s64, w64, _ = o64.export()
    err = np.abs(gs.astype(np.float64) - s64)[w64 > 0]
    assert err.max() <= (1e-5 if storage == "fp32" else 2 * seq.truncation * 2.0 ** -12)


def test_full_size_large_rooms_allocation(rf):
    """640x480 at 0.5 cm voxels, first frame (every block new), carve stride
    2: carve workgroups touch up to ~3900 distinct blocks each, more than a
    workgroup's LDS list of first touches holds, so the path that appends
    the excess to the frame list directly runs too."""
    seq = synth.large_rooms(n_frames=2)
    m = rf.Map(map_params(rf, seq, max_blocks=1 << 19))
    o32 = O.OracleMap(seq.voxel_size, seq.truncation, seq.depth_max, 255, seq.carve_stride, real_bits=32)
    for k in range(2):
        g = gpu_frame(rf, seq, k)
        m.allocate(g, dev_pose(seq.poses[k]))
        F_gpu = gpu_keyset(m.frame_blocks())
        F_orc = o32.allocate(orc_frame(seq, k), seq.poses[k])
        assert len(F_orc) > 50000
        assert np.array_equal(F_gpu, F_orc), k
    flags, nb = m.status()
    assert flags == 0 and nb == o32.num_blocks


def test_frame_list_beyond_a_listing_run(rf):
    """Eight maps allocated in one batch (the listing then gives each map 32
    workgroups, each streaming a 32nd of its buckets) on a 640x480 frame
    facing a wall at 2.5 m with 0.5 cm voxels: about 100 k blocks, more than
    32 x 2048, so at least one workgroup's range holds more marked buckets
    than its 2048-entry run in LDS and appends the rest to the frame list one
    atomic each.  Every map's frame list equals the oracle's block set."""
    from paper_1905_02082_amd import _native as N
    W, H = 640, 480
    intr = (525.0, 525.0, 319.5, 239.5)
    depth = np.full((H, W), 2500, np.uint16)
    rgb = np.random.default_rng(11).integers(0, 256, (H, W, 3), dtype=np.uint8)
    T = np.eye(4)
    T[:3, 3] = [0.013, -0.021, 0.007]
    o32 = O.OracleMap(0.005, 0.03, 3.5, 255, 2, real_bits=32)
    F_orc = o32.allocate(O.Frame(depth, rgb, *intr, depth_scale=0.001), T)
    assert len(F_orc) > 32 * 2048
    params = rf.MapParams(0.005, 0.03, 3.5, 1 << 18, 1 << 17, 255, 2, "fp32", W * H)
    sessions = [rf.Session(params, T) for _ in range(8)]
    frames = [rf.Frame.from_numpy(depth, rgb, *intr, depth_scale=0.001)] * 8
    L = N.load()
    assert L.hashmap_allocate_batch(rf._jobs(sessions, frames), 8, None) == 0
    torch.cuda.synchronize()
    for s in sessions:
        assert np.array_equal(gpu_keyset(s.map.frame_blocks()), F_orc)
        flags, nb = s.map.status()
        assert flags == 0 and nb == len(F_orc)


def test_batched_integration_beyond_a_workgroup_table(rf):
    """Eight maps allocated and integrated in one batch on a frame facing a
    wall at 2.0 m with 0.5 cm voxels (~53 k listed blocks per map): each map
    gets 192 integration workgroups, so a workgroup's share of the list
    (~275 blocks) exceeds the 256 entries it holds in LDS at a time and its
    second chunk runs too.  Two of the maps are compared with the FP32
    mirror: blocks, sdf, weight and colour bit-exact."""
    from paper_1905_02082_amd import _native as N
    W, H = 640, 480
    intr = (525.0, 525.0, 319.5, 239.5)
    depth = np.full((H, W), 2000, np.uint16)
    rgb = np.random.default_rng(12).integers(0, 256, (H, W, 3), dtype=np.uint8)
    T = np.eye(4)
    T[:3, 3] = [0.013, -0.021, 0.007]
    o32 = O.OracleMap(0.005, 0.03, 3.5, 255, 2, real_bits=32)
    fr = O.Frame(depth, rgb, *intr, depth_scale=0.001)
    F_orc = o32.allocate(fr, T)
    o32.integrate(fr, T)
    assert len(F_orc) > 256 * 192
    params = rf.MapParams(0.005, 0.03, 3.5, 1 << 18, 1 << 16, 255, 2, "fp32", W * H)
    sessions = [rf.Session(params, T) for _ in range(8)]
    frames = [rf.Frame.from_numpy(depth, rgb, *intr, depth_scale=0.001)] * 8
    L = N.load()
    assert L.hashmap_allocate_batch(rf._jobs(sessions, frames), 8, None) == 0
    assert L.integrate_frame_batch(rf._jobs(sessions, frames), 8, None) == 0
    torch.cuda.synchronize()
    km, sm, wm, cm = o32.export()
    for s in (sessions[0], sessions[7]):
        assert s.map.status() == (0, len(F_orc))
        gk, gs, gw, gc = gpu_export_sorted(s.map)
        assert np.array_equal(gk, km)
        np.testing.assert_array_equal(gs, sm.astype(np.float32))
        np.testing.assert_array_equal(gw, wm.astype(np.float32))
        np.testing.assert_array_equal(gc, cm)


def test_track_is_deterministic(rf, room):
    """Order-independent fixed-point reduction: repeated runs are bit-identical."""
    m, _, _ = integrate_teacher_forced(rf, room, range(2))
    tp = rf.TrackParams(room.levels, room.iters)
    out = []
    for _ in range(3):
        P = dev_pose(room.poses[1])
        m.track(gpu_frame(rf, room, 2), P, tp)
        out.append(P.cpu().numpy())
    assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])


def test_track_singular_plane_keeps_pose(rf):
    """A textureless fronto-parallel plane leaves 3 degrees of freedom
    unconstrained: both sides stop on the singular system and keep the pose."""
    W, H, f = 64, 48, 60.0
    depth = np.full((H, W), 1.0, np.float32)
    rgb = np.full((H, W, 3), 120, np.uint8)
    K = (f, f, (W - 1) / 2, (H - 1) / 2)
    params = rf.MapParams(0.02, 0.06, 5.0, 1 << 14, 4096, 255, 2, "fp32", W * H)
    m = rf.Map(params)
    g = rf.Frame.from_numpy(depth, rgb, *K)
    I4 = np.eye(4)
    m.allocate(g, dev_pose(I4))
    m.integrate(g, dev_pose(I4))
    o = O.OracleMap(0.02, 0.06, 5.0, 255, 2)
    fr = O.Frame(depth, rgb, *K)
    o.allocate(fr, I4)
    o.integrate(fr, I4)
    T0 = O.pose_left_update(np.r_[0.003, -0.002, 0.004, 0.0, 0.0, 0.0], I4)
    T_ref, flags, _ = o.track(fr, T0, 2, 5)
    assert flags & 2 and np.array_equal(T_ref, T0)
    P = dev_pose(T0)
    stats = torch.zeros(16, dtype=torch.float64, device="cuda")
    m.track(g, P, rf.TrackParams(2, 5), None, stats)
    iters, fl = track_stats(stats)
    assert fl & rf.RF_FLAG_TRACK_SINGULAR and iters == 0
    np.testing.assert_array_equal(P.cpu().numpy(), T0)


def test_track_out_of_range_terms_stop_the_pass(rf, room):
    """The parity room moved 60 km along x: the rotational Jacobian y x grad S
    reaches ~6e4 per pixel, so a tile's normal-equation sums exceed the 2^34
    range of the fixed-point totals.  Those terms are not dropped silently:
    the pass stops with RF_FLAG_TRACK_RANGE and keeps the pose.  The same
    scene at the origin registers without the flag."""
    far = np.eye(4)
    far[0, 3] = 6.0e4
    res = {}
    for name, off in (("origin", np.eye(4)), ("far", far)):
        m = rf.Map(map_params(rf, room))
        for k in range(2):
            g = gpu_frame(rf, room, k)
            P = dev_pose(off @ room.poses[k])
            m.allocate(g, P)
            m.integrate(g, P)
        T0 = off @ room.poses[1]
        P = dev_pose(T0)
        stats = torch.zeros(16, dtype=torch.float64, device="cuda")
        m.track(gpu_frame(rf, room, 2), P, rf.TrackParams(room.levels, room.iters), None, stats)
        iters, fl = track_stats(stats)
        res[name] = (iters, fl, P.cpu().numpy(), T0, m.status()[0])
    iters, fl, T, T0, mflags = res["origin"]
    assert fl == 0 and iters > 0 and not np.array_equal(T, T0)
    iters, fl, T, T0, mflags = res["far"]
    assert fl & rf.RF_FLAG_TRACK_RANGE and mflags & rf.RF_FLAG_TRACK_RANGE
    np.testing.assert_array_equal(T, T0)
