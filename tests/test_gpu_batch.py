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


def serving_sequences():
    """The serving mix's resolutions (320x240, 640x480 and 1280x720) plus a
    ragged one, dynamic scenes with movers in view."""
    return [synth.dynamic_room(n_frames=4, width=320, height=240, n_clusters=2, seed=11, movers="in_view"),
            synth.dynamic_room(n_frames=4, width=640, height=480, n_clusters=1, seed=12, movers="in_view"),
            synth.dynamic_room(n_frames=4, width=1280, height=720, n_clusters=3, seed=13, movers="in_view"),
            synth.dynamic_room(n_frames=4, width=77, height=53, n_clusters=1, seed=7, movers="in_view")]


def run(rf, seqs, batched, start_offsets=(0, 0, 0, 0), tp=None):
    tp, mp = tp or rf.TrackParams(2, 6), rf.MaskParams()
    sessions = [rf.Session(map_params(rf, s, max_blocks=1 << 16), s.poses[0]) for s in seqs]
    offs = list(start_offsets[:len(seqs)])
    steps = max(s.n + o for s, o in zip(seqs, offs))
    for t in range(steps):
        active = [(i, t - o) for i, o in enumerate(offs) if 0 <= t - o < seqs[i].n]
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
    staggered = run(rf, seqs, batched=True, start_offsets=(0, 2, 1, 0))
    for a, b, c in zip(alone, mixed, staggered):
        for x, y, z in zip(a, b, c):
            assert np.array_equal(x, y) and np.array_equal(x, z)
    assert all(a[6][0] == 0 for a in alone)


def test_serving_resolutions_batched_equal_alone(rf):
    """320x240, 640x480, 1280x720 and 77x53 sessions in one batch, alone and
    with staggered starts: bit-identical poses, masks and maps."""
    seqs = serving_sequences()
    alone = run(rf, seqs, batched=False)
    mixed = run(rf, seqs, batched=True)
    staggered = run(rf, seqs, batched=True, start_offsets=(0, 2, 1, 3))
    for a, b, c in zip(alone, mixed, staggered):
        for x, y, z in zip(a, b, c):
            assert np.array_equal(x, y) and np.array_equal(x, z)
    assert all(a[6][0] == 0 for a in alone)
    assert all(a[1].any() for a in alone[:3])  # the movers are masked in every size


def test_separate_solves_equal_fused_levenberg_marquardt(rf):
    """The serving mix under Levenberg-Marquardt: batched, level 0 has more
    than 3072 workgroups and solves in a launch of its own per iteration, while
    most sessions alone solve at the start of every workgroup; poses, masks
    and maps are bit-identical either way (the accept / reject state passes
    between the two schedules' launches alike)."""
    seqs = serving_sequences()
    tp = rf.TrackParams(2, 6, lm_lambda=1e-3, adaptive=True)
    alone = run(rf, seqs, batched=False, tp=tp)
    mixed = run(rf, seqs, batched=True, tp=tp)
    for a, b in zip(alone, mixed):
        for x, y in zip(a, b):
            assert np.array_equal(x, y)
    assert all(a[6][0] == 0 for a in alone)


def test_serve_loop_results_equal_alone(rf):
    """The continuous-batching loop itself: five sessions of mixed resolution
    with Poisson arrivals under a budget that admits at most two maps at a
    time (the others wait for memory).  It finishes, and each session's final
    pose and map are bit-identical to running that session alone."""
    from paper_1905_02082_amd import serving
    seqs = [synth.parity_room(n_frames=6),
            synth.dynamic_room(n_frames=6, width=160, height=120, n_clusters=2, movers="in_view"),
            synth.dynamic_room(n_frames=6, width=320, height=240, n_clusters=1, seed=11, movers="in_view"),
            synth.dynamic_room(n_frames=6, width=77, height=53, n_clusters=1, seed=7, movers="in_view"),
            synth.dynamic_room(n_frames=6, width=160, height=120, n_clusters=1, seed=5, movers="in_view")]
    tp, mp = rf.TrackParams(2, 6), rf.MaskParams()
    rng = np.random.default_rng(3)
    specs = []
    for i, sq in enumerate(seqs):
        n = 9
        order = serving.ping_pong(sq.n, n)
        arr = serving.poisson_arrivals(n, 0.01 * i, 30.0, rng)
        specs.append(serving.SessionSpec(i, sq, order, arr,
                                         map_params(rf, sq, "fp16", max_blocks=1 << 16, num_buckets=1 << 18)))
    sizes = [rf.hashmap_bytes(s.params) for s in specs]
    budget = max(sizes) * 2 + 1
    finals = {}

    def keep(spec, sess):
        keys, sdf, w, rgb = [t.cpu().numpy() for t in sess.map.export()]
        o = np.lexsort((keys[:, 2], keys[:, 1], keys[:, 0]))
        finals[spec.sid] = (sess.pose.cpu().numpy(), keys[o], sdf[o], w[o], rgb[o], sess.map.status())

    r = serving.serve(specs, tp, mp, budget, max_batch=8, depth=2, on_finish=keep)
    assert r.frames == sum(len(s.arrivals) for s in specs) and len(finals) == len(specs)
    assert r.peak_bytes <= budget and r.peak_sessions <= 2 and r.admitted_late > 0
    for spec in specs:
        sq = spec.seq
        sess = rf.Session(spec.params, sq.poses[spec.order[0]])
        for k in spec.order:
            rf.process_batch([sess], [gpu_frame(rf, sq, int(k))], tp, mp)
        torch.cuda.synchronize()
        keys, sdf, w, rgb = [t.cpu().numpy() for t in sess.map.export()]
        o = np.lexsort((keys[:, 2], keys[:, 1], keys[:, 0]))
        ref = (sess.pose.cpu().numpy(), keys[o], sdf[o], w[o], rgb[o], sess.map.status())
        for x, y in zip(finals[spec.sid], ref):
            assert np.array_equal(x, y), spec.sid


def test_serve_rejects_session_larger_than_budget(rf):
    from paper_1905_02082_amd import serving
    sq = synth.parity_room(n_frames=2)
    p = map_params(rf, sq, "fp16", max_blocks=1 << 14)
    spec = serving.SessionSpec(0, sq, np.array([0, 1]), np.array([0.0, 0.03]), p)
    with pytest.raises(ValueError):
        serving.serve([spec], rf.TrackParams(2, 2), rf.MaskParams(), rf.hashmap_bytes(p) - 1)


def test_batch_rejects_duplicate_maps(rf):
    seq = synth.parity_room(n_frames=2)
    s = rf.Session(map_params(rf, seq), seq.poses[0])
    f = gpu_frame(rf, seq, 0)
    with pytest.raises(rf.RefusionError):
        rf.process_batch([s, s], [f, f], rf.TrackParams(), rf.MaskParams())
