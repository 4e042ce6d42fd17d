"""Precision form: FP16 sdf/tau + u8 weight storage against FP32 storage and
the FP64 oracle on the same seeded inputs (teacher-forced: every frame fused
at its ground-truth pose).  The measured errors are printed and, when the
environment variable RF_RESULTS_DIR names a folder, written to
precision.json there."""
import json
import os

import numpy as np
import pytest
import torch

import oracle as O
import synth
from gpu_helpers import dev_pose, gpu_export_sorted, gpu_frame, map_params, need_gpu, orc_frame, pose_error

pytestmark = pytest.mark.gpu

N_FUSE = 10


@pytest.fixture(scope="module")
def rf():
    return need_gpu()


@pytest.fixture(scope="module")
def setup(rf):
    seq = synth.dynamic_room(n_frames=N_FUSE + 2, width=160, height=120, n_clusters=1, movers="in_view")
    maps = {st: rf.Map(map_params(rf, seq, st, max_blocks=1 << 15)) for st in ("fp32", "fp16")}
    o64 = O.OracleMap(seq.voxel_size, seq.truncation, seq.depth_max, 255, seq.carve_stride, real_bits=64)
    for k in range(N_FUSE):
        P = dev_pose(seq.poses[k])
        g = gpu_frame(rf, seq, k)
        for m in maps.values():
            m.allocate(g, P)
            m.integrate(g, P)
        o64.allocate(orc_frame(seq, k), seq.poses[k])
        o64.integrate(orc_frame(seq, k), seq.poses[k])
    torch.cuda.synchronize()
    return seq, maps, o64


def record(key, value):
    out = os.environ.get("RF_RESULTS_DIR", "")
    print("precision", key, value)
    if out and os.path.isdir(out):
        path = os.path.join(out, "precision.json")
        d = json.load(open(path)) if os.path.exists(path) else {}
        d[key] = value
        json.dump(d, open(path, "w"), indent=1)


def test_sdf_error_fp32_fp16_vs_fp64(setup):
    seq, maps, o64 = setup
    k64, s64, w64, _ = o64.export()
    tau = float(np.float32(seq.truncation))
    for st, m in maps.items():
        gk, gs, gw, _ = gpu_export_sorted(m)
        assert np.array_equal(gk, k64)
        obs = w64 > 0
        err = np.abs(gs.astype(np.float64) - s64)[obs]
        band = obs & (np.abs(s64) < tau)
        zero = obs & (np.abs(s64) < 0.25 * float(seq.voxel_size))
        e_band = np.abs(gs.astype(np.float64) - s64)[band]
        e_zero = np.abs(gs.astype(np.float64) - s64)[zero]
        record("sdf_%s_vs_fp64" % st, {"max_m": float(err.max()), "band_max_m": float(e_band.max()),
                                        "band_rms_m": float(np.sqrt(np.mean(e_band ** 2))),
                                        "near_zero_max_m": float(e_zero.max()) if e_zero.size else 0.0,
                                        "frames": N_FUSE})
        if st == "fp32":
            assert err.max() <= 1e-5
        else:
            # per store at most 2^-12 tau (half an ulp of sdf/tau in [0.5, 1)); errors decay by W/(W+1)
            assert err.max() <= N_FUSE * tau * 2.0 ** -12
        np.testing.assert_array_equal(gw, w64.astype(np.float32))


def test_pose_error_fp32_fp16_vs_fp64(rf, setup):
    seq, maps, o64 = setup
    k = N_FUSE
    T_ref, flags, _ = o64.track(orc_frame(seq, k), seq.poses[k - 1], seq.levels, seq.iters)
    assert flags == 0
    out = {}
    for st, m in maps.items():
        P = dev_pose(seq.poses[k - 1])
        m.track(gpu_frame(rf, seq, k), P, rf.TrackParams(seq.levels, seq.iters))
        dt, dr = pose_error(P.cpu().numpy(), T_ref)
        gt_t, gt_r = pose_error(P.cpu().numpy(), seq.poses[k])
        out[st] = {"vs_fp64_m": dt, "vs_fp64_rad": dr, "vs_truth_m": gt_t, "vs_truth_rad": gt_r}
        if st == "fp32":
            assert dt <= 1e-4 and dr <= 1e-5
        else:
            assert dt <= 2e-3 and dr <= 2e-4
    gt_t, gt_r = pose_error(T_ref, seq.poses[k])
    out["fp64_oracle"] = {"vs_truth_m": gt_t, "vs_truth_rad": gt_r}
    record("pose_after_%d_frames" % N_FUSE, out)
