"""compute_dynamic_mask_static (the allocation-free variant of
compute_dynamic_mask, its flood-fill scratch in a static device array)
against compute_dynamic_mask on the same inputs, through the C ABI: two
calls in a row, the second with a smaller frame, and a frame beyond the
static array's size rejected before anything runs."""
import ctypes

import numpy as np
import pytest
import torch

import synth
from gpu_helpers import dev_pose, gpu_frame, map_params, need_gpu

pytestmark = pytest.mark.gpu


def fused_map(rf, seq, frames):
    m = rf.Map(map_params(rf, seq, max_blocks=1 << 17))
    for k in frames:
        g = gpu_frame(rf, seq, k)
        P = dev_pose(seq.poses[k])
        mk = torch.from_numpy((seq.labels[k] > 0).astype(np.uint8)).cuda()
        m.allocate(g, P, mk)
        m.integrate(g, P, mk)
    return m


def both(rf, m, seq, k):
    L = rf.lib()
    g = gpu_frame(rf, seq, k)
    P = dev_pose(seq.poses[k])
    c = rf.MaskParams(0.5, 0.007).c()
    shape = (seq.height, seq.width)
    out = []
    for fn in (L.compute_dynamic_mask, L.compute_dynamic_mask_static):
        mask = torch.full(shape, 7, dtype=torch.uint8, device="cuda")
        res = torch.full(shape, 5.0, dtype=torch.float32, device="cuda")
        st = fn(m.h, ctypes.byref(g.s), ctypes.c_void_p(P.data_ptr()), ctypes.byref(c),
                ctypes.c_void_p(mask.data_ptr()), ctypes.c_void_p(res.data_ptr()), None)
        assert st == 0, rf.lib().rf_last_error()
        torch.cuda.synchronize()
        out.append((mask.cpu().numpy(), res.cpu().numpy()))
    return out


def test_static_scratch_mask_equals_arena_mask():
    rf = need_gpu()
    big = synth.dynamic_room(n_frames=8, width=320, height=240, n_clusters=2, seed=11, movers="in_view")
    small = synth.dynamic_room(n_frames=8, width=77, height=53, n_clusters=1, seed=7, movers="in_view")
    mb = fused_map(rf, big, range(0, 6, 2))
    ms = fused_map(rf, small, range(0, 6, 2))
    for m, seq in ((mb, big), (ms, small)):   # second call: a smaller frame
        (a_mask, a_res), (b_mask, b_res) = both(rf, m, seq, 7)
        assert np.array_equal(a_mask, b_mask)
        assert np.array_equal(a_res, b_res)
        assert a_mask.any() and (a_mask <= 1).all()
    # and the large one again after the small one (stale scratch must not matter)
    (a_mask, a_res), (b_mask, b_res) = both(rf, mb, big, 6)
    assert np.array_equal(a_mask, b_mask) and np.array_equal(a_res, b_res)


def test_static_scratch_rejects_oversized_frame():
    rf = need_gpu()
    seq = synth.parity_room(n_frames=1)
    m = rf.Map(map_params(rf, seq))
    W, H = 2400, 1800   # 4.3 M pixels: more than the 4 MiB static scratch holds
    depth = torch.zeros((H, W), dtype=torch.float32, device="cuda")
    rgb = torch.zeros((H, W, 3), dtype=torch.uint8, device="cuda")
    g = rf.Frame(depth, rgb, 500.0, 500.0, W / 2, H / 2)
    out = torch.zeros((H, W), dtype=torch.uint8, device="cuda")
    c = rf.MaskParams().c()
    P = dev_pose(np.eye(4))
    st = rf.lib().compute_dynamic_mask_static(m.h, ctypes.byref(g.s), ctypes.c_void_p(P.data_ptr()),
                                              ctypes.byref(c), ctypes.c_void_p(out.data_ptr()), None, None)
    assert st == rf.RF_ENOMEM if hasattr(rf, "RF_ENOMEM") else st == -2
    assert not out.any()
