"""Pins of the oracle's compact free space (the free-space representation
that Sec. III-D leaves to future work, read as coarse free-block flags; map
option free_blocks=1), against closed forms and against the per-voxel
carving of Sec. III-D (no GPU).

Reading: a block whose 8 corner voxels lie in front of the clipping plane
and project, with a one-pixel border, into a part of the image where every
8x8 cell has a measured, unmasked depth more than tau (+1 mm) beyond the
block's farthest corner is carved whole (every voxel takes the free-space
update).  A new block is a free block: no voxels, one value (sdf tau, weight
= frames that carved all of its voxels) that all its voxels read as.  A frame
that carves it whole, or carves every one of its voxels by the per-voxel
rule, adds one to the weight; a band update of any voxel turns it into a
block of voxels starting from that value; any other frame leaves it as it
is, so the value only ever stands for space observed free in every voxel."""
import numpy as np
import pytest

import oracle as O
import synth
from synth import analytic as A


def plane_frame(d, W=40, H=30, f=30.0, holes=None, color=(200, 100, 50)):
    depth = np.full((H, W), d, np.float32)
    if holes is not None:
        depth[holes] = 0.0
    rgb = np.zeros((H, W, 3), np.uint8)
    rgb[:] = color
    return O.Frame(depth, rgb, f, f, (W - 1) / 2, (H - 1) / 2)


def maps(s, tau, bits=64, dmax=5.0, stride=2, storage=0):
    return (O.OracleMap(s, tau, dmax, 255, stride, real_bits=bits, storage=storage),
            O.OracleMap(s, tau, dmax, 255, stride, real_bits=bits, storage=storage, free_blocks=1))


def voxels_by_key(m):
    keys, sdf, w, rgb = m.export()
    return {tuple(k): (sdf[i], w[i], rgb[i]) for i, k in enumerate(keys)}


def fuse(m, frames, poses, masks=None):
    out = []
    for i, (fr, T) in enumerate(zip(frames, poses)):
        mk = None if masks is None else masks[i]
        m.allocate(fr, T, mk)
        out.append(m.integrate(fr, T, mk))
    return out


@pytest.mark.parametrize("bits", [64, 32])
def test_first_frame_against_per_voxel_carving(bits):
    """With every pixel measured, after the first frame the blocks holding
    voxels are exactly those where per-voxel carving gave a voxel a band
    update, and they hold exactly the per-voxel map's voxels; every other
    listed block is a free block of weight 1 when per-voxel carving carved
    all 512 of its voxels (tau, 1) and of weight 0 otherwise (so the block
    test is sound: a block carved whole has every voxel carved)."""
    room = synth.parity_room(n_frames=3)
    fr = O.Frame(room.depth[0], room.rgb[0], *room.intrinsics)
    assert (room.depth[0] > 0).all()
    a, b = maps(room.voxel_size, room.truncation, bits, room.depth_max, room.carve_stride)
    fuse(a, [fr], [room.poses[0]])
    cnt = fuse(b, [fr], [room.poses[0]])[0]
    full = voxels_by_key(a)
    comp = voxels_by_key(b)
    fk, fw = b.export_free()
    assert len(fk) > 100 and cnt[2] > 0 and set(np.unique(fw)) <= {0.0, 1.0} and (fw == 1).sum() > 20
    assert b.num_blocks == a.num_blocks == len(comp) + len(fk)
    tau = float(np.float32(room.truncation))
    band = {k for k, (sdf, w, rgb) in full.items() if np.any((w > 0) & (sdf != tau))}
    assert band == set(comp)
    for k, (sdf, w, rgb) in comp.items():
        s2, w2, c2 = full[k]
        assert np.array_equal(sdf, s2) and np.array_equal(w, w2) and np.array_equal(rgb, c2)
    partial = 0
    for k, wk in zip(map(tuple, fk), fw):
        sdf, w, rgb = full[k]
        carved = w == 1
        assert carved.all() == (wk == 1)
        assert np.all(sdf[carved] == tau) and np.all(w[~carved] == 0) and np.all(rgb == 0)
        partial += bool(carved.any() and not carved.all())
    assert partial > 10  # partly carved blocks stay unobserved


@pytest.mark.parametrize("bits", [64, 32])
def test_free_block_reads_tau_and_counts_frames(bits):
    """A wall 1.4 m away seen n times: blocks wholly in front of it and in
    view are free blocks of weight n whose voxels read (tau, n), blocks the
    frustum's sides cut are free blocks of weight 0 (unobserved); the voxel
    blocks at the wall hold d - z in the band, as the per-voxel rule gives;
    free space costs no voxel storage."""
    s, tau, d, n = 0.02, 0.06, 1.4, 5
    a, b = maps(s, tau, bits)
    fr = plane_frame(d)
    fuse(a, [fr] * n, [np.eye(4)] * n)
    fuse(b, [fr] * n, [np.eye(4)] * n)
    fk, fw = b.export_free()
    assert (fw == n).sum() > 50 and set(np.unique(fw)) <= {0.0, float(n)}
    assert b.num_voxel_blocks + len(fk) == a.num_voxel_blocks  # free space costs no voxels
    # free blocks read tau with weight n at every voxel (through the sampler);
    # those of weight 0 read as unobserved
    full = voxels_by_key(a)
    for k, wk in zip(fk, fw):
        y = (8 * k.astype(np.float64) + 3.25) * float(np.float32(s))  # a cell inside the block
        ok, out = b.sample(y)
        assert ok == (wk == n)
        if ok:
            assert out[0] == float(np.float32(tau)) and np.all(out[1:4] == 0)
        else:
            assert not np.all(full[tuple(k)][1] == n)  # per-voxel carving did not carve it all
    # voxel blocks equal the per-voxel map (every voxel there was updated
    # identically: the same frame each time, blocks never switch)
    for k, (sdf, w, rgb) in voxels_by_key(b).items():
        assert np.array_equal(sdf, full[k][0]) and np.array_equal(w, full[k][1])
    D = float(np.float32(d))
    keys, sdf, w, _ = b.export()
    cen = A.block_voxel_centres(keys, s).reshape(-1, 3)
    band = (w.reshape(-1) == n) & (np.abs(D - cen[:, 2]) < tau - 1e-6)
    assert band.sum() > 100
    np.testing.assert_allclose(sdf.reshape(-1)[band], D - cen[band, 2], atol=1e-12 if bits == 64 else 2e-7)


def test_moved_object_still_fades():
    """A wall at 0.9 m for 4 frames, then at 1.6 m: the voxels of the old
    wall decay toward tau by the running-average recurrence, whether their
    blocks are carved whole or voxel by voxel; free blocks in front of both
    walls and wholly in view count all 7 frames, those behind the first wall
    the last 3 or none."""
    s, tau = 0.02, 0.06
    _, b = maps(s, tau)
    near, far = plane_frame(0.9), plane_frame(1.6)
    fuse(b, [near] * 4, [np.eye(4)] * 4)
    k0, sdf0, w0, _ = b.export()
    fuse(b, [far] * 3, [np.eye(4)] * 3)
    k1, sdf1, w1, _ = b.export()
    old = {tuple(k): i for i, k in enumerate(k0)}
    cen = A.block_voxel_centres(k1, s)
    checked = 0
    for i, k in enumerate(map(tuple, k1)):
        if k not in old:
            continue
        j = old[k]
        c = cen[i]
        with np.errstate(divide="ignore", invalid="ignore"):
            inside = (c[:, 2] > 0) & (np.abs(30 * c[:, 0] / c[:, 2]) < 18) & (np.abs(30 * c[:, 1] / c[:, 2]) < 13)
        was_band = (w0[j] == 4) & (np.abs(0.9 - c[:, 2]) < tau - 1e-3) & inside & (c[:, 2] < 1.6 - tau - 1e-3)
        ref = sdf0[j].copy()
        W = w0[j].copy()
        for _ in range(3):
            ref = (W * ref + float(np.float32(tau))) / (W + 1)
            W = W + 1
        np.testing.assert_allclose(sdf1[i][was_band], ref[was_band], rtol=0, atol=1e-15)
        assert np.all(w1[i][was_band] == 7)
        checked += was_band.sum()
    assert checked > 100
    fk, fw = b.export_free()
    c = A.block_voxel_centres(fk, s)
    with np.errstate(divide="ignore", invalid="ignore"):
        seen = np.all((c[:, :, 2] > 0) & (np.abs(30 * c[:, :, 0] / c[:, :, 2]) < 18)
                      & (np.abs(30 * c[:, :, 1] / c[:, :, 2]) < 13), axis=1)
    front = (c[:, :, 2].max(1) < 0.9 - tau - 0.02) & seen
    assert front.sum() > 10 and np.all(fw[front] == 7) and set(np.unique(fw)) <= {0.0, 3.0, 7.0}


def test_unmeasured_pixels_are_carved_over_masked_are_not():
    """Pixels without a measurement inside a block's image rectangle do not
    stop it being carved whole (per-voxel carving leaves the voxels that
    project onto them untouched); a masked pixel does: a block of voxels in
    free space is then carved voxel by voxel, and the voxels seen through the
    masked pixel keep their weight."""
    s, tau = 0.02, 0.06
    holes = np.zeros((30, 40), bool)
    holes[14:16, 19:21] = True
    y = np.array([0.0, 0.0, 0.6])   # in front of the hole, half-way to the wall
    a, b = maps(s, tau)
    fuse(a, [plane_frame(1.4, holes=holes)], [np.eye(4)])
    fuse(b, [plane_frame(1.4, holes=holes)], [np.eye(4)])
    ok_a, _ = a.sample(y)
    ok_b, out = b.sample(y)
    assert not ok_a            # per-voxel carving left voxels in front of the hole unobserved
    assert ok_b and out[0] == float(np.float32(tau))
    # blocks of voxels round y (a wall at 0.62 m for 3 frames), then the wall
    # at 1.4 m: carved whole without a mask, voxel by voxel with the pixels
    # round the image centre masked
    mask = holes.astype(np.uint8)
    res = []
    for mk in (None, mask):
        _, c = maps(s, tau)
        fuse(c, [plane_frame(0.62)] * 3, [np.eye(4)] * 3)
        k0 = {tuple(k) for k in c.export()[0]}
        cnt = fuse(c, [plane_frame(1.4)], [np.eye(4)], masks=[mk])[0]
        keys, sdf, w, _ = c.export()
        i = [tuple(k) for k in keys].index(tuple(np.floor(y / (8 * float(np.float32(s)))).astype(int)))
        assert tuple(keys[i]) in k0
        res.append((cnt[2], w[i]))
    (whole0, w0), (whole1, w1) = res
    assert whole1 < whole0
    assert np.all(w0 == 4)                    # carved whole: every voxel updated
    assert (w1 == 3).sum() > 0 and (w1 == 4).sum() > 0   # masked pixels: those voxels untouched


def test_clipping_plane_bounds_free_space():
    """A wall beyond the clipping plane (1.8 m, plane 1.0 m) adds no band, so
    no block takes voxels, and the carve rays end at the plane: every listed
    block lies in front of it and, seen twice from the same pose, has weight
    2 (a voxel carved in each frame) or 0 (none)."""
    s, tau = 0.02, 0.06
    _, b = maps(s, tau, dmax=1.0)
    fuse(b, [plane_frame(1.8)] * 2, [np.eye(4)] * 2)
    fk, fw = b.export_free()
    z = A.block_voxel_centres(fk, s)[:, :, 2]
    assert b.num_voxel_blocks == 0 and len(fk) > 50
    assert np.all(z.min(1) <= 1.0 + 1e-6)
    assert set(np.unique(fw)) <= {0.0, 2.0} and (fw == 2).sum() > 50


def test_free_block_becomes_voxels_starting_from_its_value():
    """Free blocks in front of a wall at 1.6 m (3 frames), then a wall at
    1.2 m: the blocks the new wall cuts become voxel blocks whose voxels start
    from their free value: from (tau, 3), so a band voxel holds
    (3 tau + (d - z)) / 4 and weight 4, when all their voxels were carved in
    each frame, and from unobserved, so a band voxel holds d - z and weight
    1, when the frustum's sides cut them."""
    s, tau = 0.02, 0.06
    _, b = maps(s, tau)
    fuse(b, [plane_frame(1.6)] * 3, [np.eye(4)] * 3)
    fk3, fw3 = b.export_free()
    assert set(np.unique(fw3)) <= {0.0, 3.0}
    weight = {tuple(k): wk for k, wk in zip(fk3, fw3)}
    fuse(b, [plane_frame(1.2)], [np.eye(4)])
    keys, sdf, w, _ = b.export()
    cen = A.block_voxel_centres(keys, s)
    D, T = float(np.float32(1.2)), float(np.float32(tau))
    checked = [0, 0]
    for i, k in enumerate(map(tuple, keys)):
        if k not in weight:
            continue
        c = cen[i]
        n = int(weight[k])
        band = (np.abs(D - c[:, 2]) < tau - 1e-6) & (w[i] == n + 1)
        ref = (n * T + (D - c[:, 2])) / (n + 1)
        np.testing.assert_allclose(sdf[i][band], ref[band], rtol=0, atol=1e-15)
        checked[n == 3] += band.sum()
    assert checked[0] > 20 and checked[1] > 50


def test_block_behind_a_silhouette_keeps_its_occluded_voxels_unobserved():
    """A near half-plane (0.6 m, left) in front of a far one (1.6 m, right):
    blocks behind the near half's edge are carved through the right-hand
    pixels and occluded through the left-hand ones.  No voxel behind the
    surface may read as free: such a block, unless a voxel of it is in the
    band (then it holds exactly the per-voxel voxels), stays a free block of
    weight 0, its carved voxels unrecorded, and reads as unobserved; seen
    again from the side that carves it all, it counts that frame."""
    s, tau = 0.02, 0.06
    W, H, f = 40, 30, 30.0
    depth = np.full((H, W), 1.6, np.float32)
    depth[:, :23] = 0.6
    rgb = np.full((H, W, 3), 90, np.uint8)
    fr = O.Frame(depth, rgb, f, f, (W - 1) / 2, (H - 1) / 2)
    a, b = maps(s, tau)
    fuse(a, [fr], [np.eye(4)])
    fuse(b, [fr], [np.eye(4)])
    full, comp = voxels_by_key(a), voxels_by_key(b)
    mixed = []
    for k in full:
        c = A.block_voxel_centres(np.array([k]), s)[0]
        with np.errstate(divide="ignore", invalid="ignore"):
            u = np.floor(f * c[:, 0] / c[:, 2] + (W - 1) / 2 + 0.5)
            v = np.floor(f * c[:, 1] / c[:, 2] + (H - 1) / 2 + 0.5)
        inside = (c[:, 2] > 0) & (u >= 0) & (u < W) & (v >= 0) & (v < H)
        occluded = inside & (u < 23) & (c[:, 2] > 0.6 + tau + 1e-3)
        carved = inside & (u >= 23) & (c[:, 2] < 1.6 - tau - 1e-3)
        if occluded.any() and carved.any():
            mixed.append(k)
    assert len(mixed) > 3
    fk, fw = b.export_free()
    free_w = {tuple(q): wq for q, wq in zip(fk, fw)}
    n_free = 0
    for k in mixed:
        if k in comp:
            assert np.array_equal(comp[k][1], full[k][1]) and np.array_equal(comp[k][0], full[k][0])
        else:
            assert free_w[k] == 0
            y = (8 * np.array(k, np.float64) + 3.25) * float(np.float32(s))
            assert not b.sample(y)[0]
            n_free += 1
    assert n_free > 3
    # with the near half gone every voxel of those blocks is carved
    far = O.Frame(np.full((H, W), 1.6, np.float32), rgb, f, f, (W - 1) / 2, (H - 1) / 2)
    fuse(b, [far], [np.eye(4)])
    fk, fw = b.export_free()
    free_w = {tuple(q): wq for q, wq in zip(fk, fw)}
    def wholly_carved(k):
        c = A.block_voxel_centres(np.array([k]), s)[0]
        if not np.all((c[:, 2] > 0) & (c[:, 2] < 1.6 - tau - 1e-3)):
            return False
        u = f * c[:, 0] / c[:, 2] + (W - 1) / 2
        v = f * c[:, 1] / c[:, 2] + (H - 1) / 2
        return bool(np.all((u > -0.4) & (u < W - 0.6) & (v > -0.4) & (v < H - 0.6)))
    inner = [k for k in mixed if k not in comp and wholly_carved(k)]
    assert len(inner) > 0 and all(free_w[k] == 1 for k in inner)
