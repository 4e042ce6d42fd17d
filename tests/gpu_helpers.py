"""Helpers for GPU-vs-oracle parity tests (inputs from synth/, expected
values only from oracle/)."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle as O


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1905_02082_amd as rf
    rf.lib()  # raises if the HIP library is not built
    return rf


def dev_pose(T):
    return torch.as_tensor(np.asarray(T, np.float64)).cuda().contiguous()


def gpu_frame(rf, seq, k):
    return rf.Frame.from_numpy(seq.depth[k], seq.rgb[k], *seq.intrinsics, depth_scale=seq.depth_scale)


def orc_frame(seq, k):
    return O.Frame(seq.depth[k], seq.rgb[k], *seq.intrinsics, depth_scale=seq.depth_scale)


def map_params(rf, seq, storage="fp32", max_blocks=None, num_buckets=None):
    return rf.MapParams(seq.voxel_size, seq.truncation, seq.depth_max, num_buckets or seq.num_buckets,
                        max_blocks or (1 << 16), 255, seq.carve_stride, storage, seq.width * seq.height)


def oracle_maps(seq, storage=0):
    """(FP64 reference, FP32 mirror) oracle maps with the sequence's parameters."""
    a = O.OracleMap(seq.voxel_size, seq.truncation, seq.depth_max, 255, seq.carve_stride, real_bits=64)
    b = O.OracleMap(seq.voxel_size, seq.truncation, seq.depth_max, 255, seq.carve_stride, real_bits=32,
                    storage=storage)
    return a, b


def sort_keys(keys):
    keys = np.asarray(keys, np.int64).reshape(-1, 3)
    order = np.lexsort((keys[:, 2], keys[:, 1], keys[:, 0]))
    return order


def gpu_export_sorted(m):
    keys, sdf, w, rgb = [t.cpu().numpy() for t in m.export()]
    o = sort_keys(keys)
    return keys[o], sdf[o], w[o], rgb[o]


def gpu_keyset(keys_tensor):
    k = keys_tensor.cpu().numpy()
    return k[sort_keys(k)]


def pose_error(Ta, Tb):
    dt = float(np.linalg.norm(Ta[:3, 3] - Tb[:3, 3]))
    R = Ta[:3, :3].T @ Tb[:3, :3]
    dr = float(np.arccos(np.clip((np.trace(R) - 1) / 2, -1.0, 1.0)))
    return dt, dr
