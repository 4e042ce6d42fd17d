"""A recorded frame step (GraphStep, HIP graph replay) does exactly what eager
steps do: every replay is checked against an eager session bit for bit, with
eager work and host synchronisations between the replays, for one session and
for a batch of two."""
import numpy as np
import pytest
import torch

import synth
from gpu_helpers import gpu_frame, map_params, need_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rf():
    return need_gpu()


def snapshot(s):
    keys, sdf, w, rgb = [t.cpu().numpy() for t in s.map.export()]
    o = np.lexsort((keys[:, 2], keys[:, 1], keys[:, 0]))
    return [s.pose.cpu().numpy(), s.mask.cpu().numpy(), s.stats.cpu().numpy(), keys[o], sdf[o], w[o], rgb[o],
            np.asarray(s.map.status())]


@pytest.mark.parametrize("split", [False, True])
def test_graph_replays_equal_eager_steps(rf, split):
    seqs = [synth.dynamic_room(n_frames=8, width=160, height=120, n_clusters=2, movers="in_view"),
            synth.dynamic_room(n_frames=8, width=160, height=120, n_clusters=1, seed=5, movers="in_view")]
    tp, mp = rf.TrackParams(2, 5), rf.MaskParams()
    eager = [rf.Session(map_params(rf, s, max_blocks=1 << 15), s.poses[0]) for s in seqs]
    graph = [rf.Session(map_params(rf, s, max_blocks=1 << 15), s.poses[0]) for s in seqs]
    for batch in ([0], [0, 1]):
        es, gs = [eager[i] for i in batch], [graph[i] for i in batch]
        first = gs[0].k
        step = None
        for k in range(first, first + 4):
            frames = [gpu_frame(rf, seqs[i], k) for i in batch]
            rf.process_batch(es, frames, tp, mp)
            if gs[0].k == 0:
                rf.process_batch(gs, frames, tp, mp)
                continue
            if step is None:
                step = rf.GraphStep(gs, frames, tp, mp, split=split)
            step(frames)
            torch.cuda.synchronize()
            for a, b in zip(es, gs):
                for x, y in zip(snapshot(a), snapshot(b)):
                    assert np.array_equal(x, y), (batch, k)
        if batch == [0]:
            # bring session 1 to the same frame eagerly before the batch of two
            for k in range(first + 4):
                frames = [gpu_frame(rf, seqs[1], k)]
                rf.process_batch([eager[1]], frames, tp, mp)
                rf.process_batch([graph[1]], frames, tp, mp)


def test_graph_step_rejects_first_frame_and_other_sizes(rf):
    seq = synth.parity_room(n_frames=3)
    tp, mp = rf.TrackParams(1, 2), rf.MaskParams()
    s = rf.Session(map_params(rf, seq), seq.poses[0])
    f0 = gpu_frame(rf, seq, 0)
    with pytest.raises(rf.RefusionError):
        rf.GraphStep([s], [f0], tp, mp)
    rf.process_batch([s], [f0], tp, mp)
    step = rf.GraphStep([s], [gpu_frame(rf, seq, 1)], tp, mp)
    other = synth.dynamic_room(n_frames=1, width=77, height=53, n_clusters=1, movers="in_view")
    with pytest.raises(rf.RefusionError):
        step([gpu_frame(rf, other, 0)])
    torch.cuda.synchronize()


def test_pipeline_graph_mode_equals_eager(rf):
    seq = synth.dynamic_room(n_frames=6, width=160, height=120, n_clusters=2, movers="in_view")
    tp, mp = rf.TrackParams(2, 5), rf.MaskParams()
    a = rf.Pipeline(map_params(rf, seq, max_blocks=1 << 15), tp, mp, seq.poses[0])
    b = rf.Pipeline(map_params(rf, seq, max_blocks=1 << 15), tp, mp, seq.poses[0], graph=True)
    for k in range(seq.n):
        f = gpu_frame(rf, seq, k)
        a.process(f)
        b.process(f)
    torch.cuda.synchronize()
    for x, y in zip(snapshot(a.session), snapshot(b.session)):
        assert np.array_equal(x, y)
