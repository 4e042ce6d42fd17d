"""Batched (multi-session) execution: every session's result is bit-identical
to processing it alone, for sessions of different resolutions in one batch."""
import numpy as np
import pytest
import torch

import synth
from gpu_helpers import gpu_frame, map_params, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rf():
    return need_gpu()


def sequences():
    return [synth.parity_room(n_frames=5),
            synth.dynamic_room(n_frames=5, width=160, height=120, n_clusters=2, movers="in_view"),
            synth.dynamic_room(n_frames=5, width=77, height=53, n_clusters=1, seed=7, movers="in_view")]


def run(rf, seqs, batched, start_offsets=(0, 0, 0)):
    tp, mp = rf.TrackParams(2, 6), rf.MaskParams()
    sessions = [rf.Session(map_params(rf, s, max_blocks=1 << 15), s.poses[0]) for s in seqs]
    steps = max(s.n + o for s, o in zip(seqs, start_offsets))
    for t in range(steps):
        active = [(i, t - o) for i, o in enumerate(start_offsets) if 0 <= t - o < seqs[i].n]
        frames = [gpu_frame(rf, seqs[i], k) for i, k in active]
        if batched:
            rf.process_batch([sessions[i] for i, _ in active], frames, tp, mp)
        else:
            for (i, _), f in zip(active, frames):
                rf.process_batch([sessions[i]], [f], tp, mp)
    torch.cuda.synchronize()
    out = []
    for s in sessions:
        keys, sdf, w, rgb = [t.cpu().numpy() for t in s.map.export()]
        o = np.lexsort((keys[:, 2], keys[:, 1], keys[:, 0]))
        out.append((s.pose.cpu().numpy(), s.mask.cpu().numpy(), keys[o], sdf[o], w[o], rgb[o], s.map.status()))
    return out


def test_batched_equals_alone(rf):
    seqs = sequences()
    alone = run(rf, seqs, batched=False)
    mixed = run(rf, seqs, batched=True)
    staggered = run(rf, seqs, batched=True, start_offsets=(0, 2, 1))
    for a, b, c in zip(alone, mixed, staggered):
        for x, y, z in zip(a, b, c):
            assert np.array_equal(x, y) and np.array_equal(x, z)
    assert all(a[6][0] == 0 for a in alone)


def test_batch_rejects_duplicate_maps(rf):
    seq = synth.parity_room(n_frames=2)
    s = rf.Session(map_params(rf, seq), seq.poses[0])
    f = gpu_frame(rf, seq, 0)
    with pytest.raises(rf.RefusionError):
        rf.process_batch([s, s], [f, f], rf.TrackParams(), rf.MaskParams())
