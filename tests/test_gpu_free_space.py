"""Compact free space (rf_map_params.free_blocks = 1; the free-space
representation Sec. III-D leaves to future work, read as coarse free-block
flags) on the GPU against the oracle's compact-free-space mirror: blocks
holding voxels bit-exact, free blocks (keys and weights) identical, and every
reader of the map -- tracking, the residual mask, the ray cast -- reading a
free block's voxels as (tau, count) exactly as the oracle does."""
import numpy as np
import pytest
import torch

import oracle as O
import synth
from gpu_helpers import (dev_pose, gpu_export_sorted, gpu_frame, map_params, need_gpu, orc_frame, pose_error,
                         sort_keys)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rf():
    return need_gpu()


def compact_params(rf, seq, storage="fp32", max_blocks=1 << 16, num_buckets=None):
    p = map_params(rf, seq, storage, max_blocks=max_blocks, num_buckets=num_buckets)
    p.free_blocks = True
    return p


def compact_oracles(seq, storage=0):
    a = O.OracleMap(seq.voxel_size, seq.truncation, seq.depth_max, 255, seq.carve_stride, real_bits=64,
                    free_blocks=1)
    b = O.OracleMap(seq.voxel_size, seq.truncation, seq.depth_max, 255, seq.carve_stride, real_bits=32,
                    storage=storage, free_blocks=1)
    return a, b


def fuse_both(rf, seq, frames, storage="fp32", orc_storage=0, masks=None, max_blocks=1 << 16):
    m = rf.Map(compact_params(rf, seq, storage, max_blocks))
    o64, o32 = compact_oracles(seq, orc_storage)
    counts = []
    for i, k in enumerate(frames):
        mk = None if masks is None else masks[i]
        g, P = gpu_frame(rf, seq, k), dev_pose(seq.poses[k])
        mt = None if mk is None else torch.from_numpy(mk).cuda()
        m.allocate(g, P, mt)
        m.integrate(g, P, mt)
        for o in (o64, o32):
            o.allocate(orc_frame(seq, k), seq.poses[k], mk)
            c = o.integrate(orc_frame(seq, k), seq.poses[k], mk)
        counts.append(c)
    torch.cuda.synchronize()
    return m, o64, o32, counts


def assert_compact_match(m, om):
    gk, gs, gw, gc = gpu_export_sorted(m)
    k, s, w, c = om.export()
    assert np.array_equal(gk, k)
    np.testing.assert_array_equal(gs, s.astype(np.float32))
    np.testing.assert_array_equal(gw, w.astype(np.float32))
    np.testing.assert_array_equal(gc, c)
    fk, fw = [t.cpu().numpy() for t in m.export_free()]
    o = sort_keys(fk)
    ok, ow = om.export_free()
    assert np.array_equal(fk[o], ok)
    np.testing.assert_array_equal(fw[o], ow.astype(np.float32))
    assert m.num_keys() == om.num_blocks
    return len(gk), len(fk)


@pytest.mark.parametrize("storage,orc_storage", [("fp32", 0), ("fp16", 1)])
def test_parity_room_compact_maps_match_mirror(rf, storage, orc_storage):
    room = synth.parity_room()
    m, o64, o32, counts = fuse_both(rf, room, range(0, 10, 2), storage, orc_storage)
    nvox, nfree = assert_compact_match(m, o32)
    assert nfree > 20 and nvox > 20
    # whole-carved blocks counted like the oracle (band / free updates too)
    assert m.cumulative_counts()[4] == sum(int(c[2]) for c in counts)
    assert m.stats_counts() == (int(counts[-1][0]), int(counts[-1][1]))


def test_dynamic_room_with_dropout_and_masks(rf):
    """640x480 dynamic room (2% unmeasured pixels carved over, masked movers
    stop whole-block carving), four frames at ground-truth poses."""
    seq = synth.dynamic_room(n_frames=8, movers="in_view")
    ks = [0, 2, 4, 6]
    masks = [(seq.labels[k] > 0).astype(np.uint8) for k in ks]
    m, o64, o32, counts = fuse_both(rf, seq, ks, masks=masks, max_blocks=1 << 17)
    nvox, nfree = assert_compact_match(m, o32)
    assert nfree > 1000 and sum(int(c[2]) for c in counts) > 5000


def test_large_rooms_compact_first_frames(rf):
    """0.5 cm voxels, 2^22 buckets, two frames: most listed blocks are free
    blocks; free space takes no pool slots."""
    seq = synth.large_rooms(n_frames=2)
    m, o64, o32, counts = fuse_both(rf, seq, range(2), max_blocks=1 << 18)
    nvox, nfree = assert_compact_match(m, o32)
    assert nfree > nvox


def test_readers_of_a_compact_map(rf):
    """Tracking, the residual mask and the ray cast read free blocks as
    (tau, count): normal equations, residuals, masks and virtual depths
    bit-exact against the mirror, poses against the FP64 compact oracle."""
    seq = synth.dynamic_room(n_frames=14, width=160, height=120, n_clusters=2, movers="in_view")
    ks = list(range(0, 12, 2))
    masks = [(seq.labels[k] > 0).astype(np.uint8) for k in ks]
    m, o64, o32, _ = fuse_both(rf, seq, ks, masks=masks)
    k = 13
    g, fr = gpu_frame(rf, seq, k), orc_frame(seq, k)
    ne = m.normal_equations(g, dev_pose(seq.poses[12]), 0, 0.025).cpu().numpy()
    ne32 = o32.normal_equations(fr, seq.poses[12], 0, 0.025)
    assert ne[28] == ne32[28] and ne[28] > 1000
    assert np.max(np.abs(ne[:28] - ne32[:28])) <= 1e-12 * np.abs(ne32[:28]).max() * ne[28]
    res = torch.empty((seq.height, seq.width), dtype=torch.float32, device="cuda")
    out = m.dynamic_mask(g, dev_pose(seq.poses[k]), rf.MaskParams(0.5, 0.007), residual=res, stages=True)
    ref = o32.mask(fr, seq.poses[k], 0.5, 0.007)
    np.testing.assert_array_equal(res.cpu().numpy(), ref["residual"])
    for key in ("raw", "eroded", "filled", "final"):
        assert np.array_equal(out[key].cpu().numpy(), ref[key]), key
    vd = m.raycast(g, dev_pose(seq.poses[k]), only_invalid=False).cpu().numpy()
    vref = o32.raycast(fr, seq.poses[k], 0.3, seq.depth_max, seq.depth_max, only_invalid=False)
    np.testing.assert_array_equal(vd, vref.astype(np.float32))
    tp = rf.TrackParams(seq.levels, seq.iters)
    P = dev_pose(seq.poses[12])
    m.track(g, P, tp)
    T, fl, _ = o64.track(fr, seq.poses[12], seq.levels, seq.iters)
    assert fl == 0
    dt, dr = pose_error(P.cpu().numpy(), T)
    assert dt <= 1e-4 and dr <= 1e-5, (dt, dr)


def test_free_running_compact_pipeline(rf):
    """The whole method per frame on a compact map (registration, mask,
    masked registration, allocation, integration), free-running over the
    160x120 parity room, against the FP64 compact oracle pipeline."""
    room = synth.parity_room()
    pipe = rf.Pipeline(compact_params(rf, room), rf.TrackParams(room.levels, room.iters), rf.MaskParams(),
                       room.poses[0], dynamic=True)
    o64, o32 = compact_oracles(room)
    T = room.poses[0]
    for k in range(room.n):
        pipe.process(gpu_frame(rf, room, k))
        T, _ = O.process_frame(o64, orc_frame(room, k), T, k, room.levels, room.iters, mask_map=o32)
        dt, dr = pose_error(pipe.pose.cpu().numpy(), T)
        assert dt <= 1e-4 and dr <= 1e-5, (k, dt, dr)
    assert pipe.map.status()[0] == 0


def test_compact_map_rejects_big_tables_and_frames(rf):
    room = synth.parity_room(n_frames=1)
    p = compact_params(rf, room, num_buckets=1 << 23)
    with pytest.raises(rf.RefusionError):
        rf.Map(p)
    p = compact_params(rf, room)
    p.max_pixels = 100
    m = rf.Map(p)
    g = gpu_frame(rf, room, 0)
    with pytest.raises(rf.RefusionError):
        m.integrate(g, dev_pose(room.poses[0]))
