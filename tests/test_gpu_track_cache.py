"""The tracking block cache (per level and tile, in the map's arena) never
changes a result: tracking with warm caches, after a reset, and after new
blocks were allocated (absent-block entries of an older allocation epoch)
gives bit for bit what a fresh map gives."""
import numpy as np
import pytest
import torch

import synth
from gpu_helpers import gpu_frame, map_params, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rf():
    return need_gpu()


def build(rf, m, seq, frames):
    for k in frames:
        P = torch.as_tensor(seq.poses[k]).cuda().contiguous()
        f = gpu_frame(rf, seq, k)
        m.allocate(f, P)
        m.integrate(f, P)


def track(rf, m, seq, k, start):
    P = torch.as_tensor(seq.poses[start]).cuda().contiguous()
    stats = torch.zeros(16, dtype=torch.float64, device="cuda")
    m.track(gpu_frame(rf, seq, k), P, rf.TrackParams(3, 6), stats=stats)
    torch.cuda.synchronize()
    return P.cpu().numpy(), stats.cpu().numpy()


@pytest.mark.parametrize("storage", ["fp32", "fp16"])
def test_block_cache_never_changes_results(rf, storage):
    seq = synth.static_room(n_frames=9, width=320, height=240)
    mp = map_params(rf, seq, storage=storage, max_blocks=1 << 16)
    warm = rf.Map(mp)
    build(rf, warm, seq, range(6))
    cold_pose, cold_stats = track(rf, warm, seq, 6, 5)      # first call: caches fill level by level
    for _ in range(2):                                      # warm caches
        p, st = track(rf, warm, seq, 6, 5)
        assert np.array_equal(p, cold_pose) and np.array_equal(st, cold_stats)
    fresh = rf.Map(mp)
    build(rf, fresh, seq, range(6))
    p, st = track(rf, fresh, seq, 6, 5)
    assert np.array_equal(p, cold_pose) and np.array_equal(st, cold_stats)
    # new blocks: the absent-block entries the caches hold are of an older epoch
    build(rf, warm, seq, [6])
    build(rf, fresh, seq, [6])
    other = rf.Map(mp)
    build(rf, other, seq, range(7))
    a = track(rf, warm, seq, 7, 6)
    b = track(rf, fresh, seq, 7, 6)
    c = track(rf, other, seq, 7, 6)
    for x, y, z in zip(a, b, c):
        assert np.array_equal(x, z) and np.array_equal(y, z)
    # a reset clears the caches (slots of the rebuilt map differ)
    warm.L.hashmap_reset(warm.h, None)
    build(rf, warm, seq, range(3, 7))
    ref = rf.Map(mp)
    build(rf, ref, seq, range(3, 7))
    for x, y in zip(track(rf, warm, seq, 7, 6), track(rf, ref, seq, 7, 6)):
        assert np.array_equal(x, y)
