"""Host-side measurement logic of bench.py (CPU): the tracking sweep's
algorithmic bytes against a brute-force count, and the rule that a committed
PMC summary is used only for the same workload and kernel source."""
import json
import types

import numpy as np
import pytest

import bench


def tiny_sequence(seed=3):
    rng = np.random.default_rng(seed)
    W, H, levels = 24, 18, 2
    depth = rng.uniform(0.5, 2.2, (H, W)).astype(np.float32)
    depth[rng.random((H, W)) < 0.1] = 0.0           # unmeasured
    depth[rng.random((H, W)) < 0.05] = 3.5          # beyond the clipping plane
    c, s_ = np.cos(0.3), np.sin(0.3)
    T = np.eye(4)
    T[:3, :3] = [[c, 0.0, s_], [0.0, 1.0, 0.0], [-s_, 0.0, c]]
    T[:3, 3] = [-0.37, 0.11, 0.23]                  # negative coordinates exercise floor division
    return types.SimpleNamespace(width=W, height=H, levels=levels, depth=[depth], depth_scale=1.0,
                                 poses=[T], intrinsics=(20.0, 20.0, 11.5, 8.5), depth_max=3.0,
                                 voxel_size=0.02)


def brute_force(seq, blocks, rec):
    """Per level: distinct allocated corner voxels x rec + distinct corner
    blocks x 16 + every pixel of the level x 5 + 29 x 8, by plain loops."""
    fx, fy, cx, cy = seq.intrinsics
    D, T = seq.depth[0].astype(np.float64), seq.poses[0]
    out = []
    for lv in range(seq.levels):
        st = 1 << lv
        voxels, corner_blocks, npix = set(), set(), 0
        for v in range(0, seq.height, st):
            for u in range(0, seq.width, st):
                npix += 1
                d = D[v, u]
                if not (0.0 < d <= seq.depth_max):
                    continue
                x = np.array([(u - cx) / fx * d, (v - cy) / fy * d, d])
                y = T[:3, :3] @ x + T[:3, 3]
                g = [int(np.floor(y[a] / seq.voxel_size)) for a in range(3)]
                for i in range(8):
                    vox = (g[0] + (i & 1), g[1] + ((i >> 1) & 1), g[2] + (i >> 2))
                    blk = tuple(c // 8 for c in vox)
                    corner_blocks.add(blk)
                    if blk in blocks:
                        voxels.add(vox)
        out.append(len(voxels) * rec + len(corner_blocks) * 16 + npix * 5 + 29 * 8)
    return out


@pytest.mark.parametrize("storage,rec", [("fp32", 12), ("fp16", 8)])
def test_track_footprint_matches_brute_force(storage, rec):
    seq = tiny_sequence()
    # every corner block the frame touches, then keep a seeded half of them
    # allocated, so the allocated-voxel filter decides part of the count
    all_blocks = set()
    fx, fy, cx, cy = seq.intrinsics
    D, T = seq.depth[0].astype(np.float64), seq.poses[0]
    for v in range(seq.height):
        for u in range(seq.width):
            d = D[v, u]
            if 0.0 < d <= seq.depth_max:
                y = T[:3, :3] @ np.array([(u - cx) / fx * d, (v - cy) / fy * d, d]) + T[:3, 3]
                g = np.floor(y / seq.voxel_size).astype(int)
                for i in range(8):
                    all_blocks.add(tuple((g + [i & 1, (i >> 1) & 1, i >> 2]) // 8))
    rng = np.random.default_rng(5)
    blocks = {b for b in sorted(all_blocks) if rng.random() < 0.5}
    assert 0 < len(blocks) < len(all_blocks)
    got, pix = bench.track_footprint(seq, np.array(sorted(blocks), dtype=np.int64).reshape(-1, 3), [0], storage)
    assert list(got) == brute_force(seq, blocks, rec)
    assert list(pix) == [seq.width * seq.height, ((seq.width + 1) // 2) * ((seq.height + 1) // 2)]


def test_traffic_from_profile_only_for_same_workload_and_source(tmp_path, monkeypatch):
    from paper_1905_02082_amd.profiling import kernel_source_hash
    key = bench.profile_key("large_rooms", 1000, "fp32", 3.5, 20)
    assert key == "large_rooms:1000 frames:fp32:depth_max 3.5:last 20 timed"
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    path = tmp_path / "profiles" / "track_large_rooms_fp32_pmc.json"
    assert bench.traffic_from_profile("track_kernel", key) == (None, None)  # no summary
    rec = {"kernel": "track_kernel", "hbm_bytes_per_launch": 123456, "l2_hit_rate": 0.5, "workload": key,
           "kernel_source_hash": kernel_source_hash("track_kernel")}
    path.write_text(json.dumps(rec))
    assert bench.traffic_from_profile("track_kernel", key) == (123456, 0.5)
    other = bench.profile_key("large_rooms", 1000, "fp32", 3.5, 100)
    assert bench.traffic_from_profile("track_kernel", other) == (None, None)  # other timed frames
    path.write_text(json.dumps(dict(rec, kernel_source_hash="0" * 16)))
    assert bench.traffic_from_profile("track_kernel", key) == (None, None)  # other kernel source
