"""Mesh extraction (marching tetrahedra) through the C ABI against the oracle:
bit-exact against the FP32 mirror (triangles compared as sorted lists), close
to the FP64 reference, on an analytic sphere map and on maps fused from
frames (FP32 and FP16 storage); capacity overflow and the empty map."""
import ctypes

import numpy as np
import pytest
import torch

import oracle as O
import synth
from gpu_helpers import dev_pose, gpu_frame, map_params, need_gpu, orc_frame, oracle_maps
from synth import analytic as A

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rf():
    return need_gpu()


def sorted_tris(T):
    T = np.asarray(T, np.float64).reshape(len(T), 9)
    return T[np.lexsort(T.T[::-1])]


def sphere_inputs(c, r, s=0.01, tau=0.05):
    ang = np.linspace(0, 2 * np.pi, 90)
    pol = np.linspace(0, np.pi, 45)
    pts = c + r * np.array([[np.cos(a) * np.sin(b), np.sin(a) * np.sin(b), np.cos(b)] for a in ang for b in pol])
    keys = A.blocks_near(pts, s, 1)
    return A.fill_map(keys, s, lambda x: np.clip(np.linalg.norm(x - c, axis=-1) - r, -tau, tau))


def test_mesh_of_analytic_sphere_matches_oracle(rf):
    s, tau = 0.01, 0.05
    c, r = np.array([0.013, -0.007, 0.021]), 0.17
    keys, sdf, w, rgb = sphere_inputs(c, r, s, tau)
    mp = rf.MapParams(s, tau, 5.0, 1 << 16, 1 << 14, 255, 4, "fp32", 64 * 64)
    m = rf.Map(mp)
    m.import_(torch.from_numpy(keys).cuda(), torch.from_numpy(sdf.astype(np.float32)).cuda(),
              torch.from_numpy(w.astype(np.float32)).cuda(), torch.from_numpy(rgb).cuda())
    g = m.mesh().cpu().numpy()
    o32 = O.OracleMap(s, tau, 5.0, 255, 4, real_bits=32)
    o32.import_(keys, sdf.astype(np.float32).astype(np.float64), w, rgb)
    o64 = O.OracleMap(s, tau, 5.0, 255, 4, real_bits=64)
    o64.import_(keys, sdf.astype(np.float32).astype(np.float64), w, rgb)
    t32, t64 = o32.mesh(), o64.mesh()
    assert len(g) == len(t32) == len(t64) > 10000
    a, b = sorted_tris(g), sorted_tris(t32)
    assert np.array_equal(a, b)                                   # bit-exact vs the FP32 mirror
    assert np.abs(t64 - t32).max() < 1e-6                         # FP64 reference, same emission order
    V = g.reshape(-1, 3).astype(np.float64)
    assert np.abs(np.linalg.norm(V - c, axis=1) - r).max() < 3 * s * s / (8 * r) * 1.01 + 1e-6


@pytest.mark.parametrize("storage,orc_storage", [("fp32", 0), ("fp16", 1)])
def test_mesh_of_fused_map_matches_mirror(rf, storage, orc_storage):
    seq = synth.parity_room(n_frames=4)
    m = rf.Map(map_params(rf, seq, storage))
    o64, o32 = oracle_maps(seq, orc_storage)
    for k in range(4):
        g = gpu_frame(rf, seq, k)
        P = dev_pose(seq.poses[k])
        m.allocate(g, P)
        m.integrate(g, P)
        fr = orc_frame(seq, k)
        for o in (o64, o32):
            o.allocate(fr, seq.poses[k])
            o.integrate(fr, seq.poses[k])
    torch.cuda.synchronize()
    gm = m.mesh().cpu().numpy()
    t32 = o32.mesh()
    assert len(gm) == len(t32) > 1000
    assert np.array_equal(sorted_tris(gm), sorted_tris(t32))
    t64 = o64.mesh()
    # the FP64 map differs from the FP32 one by rounding, so compare the
    # surfaces: every GPU vertex lies within a voxel of the FP64 mesh's vertices
    from scipy.spatial import cKDTree
    d, _ = cKDTree(t64.reshape(-1, 3)).query(gm.reshape(-1, 3).astype(np.float64))
    assert np.percentile(d, 99) < 1e-3 and d.max() < seq.voxel_size


def test_mesh_capacity_overflow_and_empty_map(rf):
    s, tau = 0.01, 0.05
    keys, sdf, w, rgb = sphere_inputs(np.zeros(3), 0.08, s, tau)
    mp = rf.MapParams(s, tau, 5.0, 1 << 14, 1 << 12, 255, 4, "fp32", 64 * 64)
    empty = rf.Map(mp)
    assert empty.mesh().shape[0] == 0
    m = rf.Map(mp)
    m.import_(torch.from_numpy(keys).cuda(), torch.from_numpy(sdf.astype(np.float32)).cuda(),
              torch.from_numpy(w.astype(np.float32)).cuda(), torch.from_numpy(rgb).cuda())
    full = m.mesh().cpu().numpy()
    cap = len(full) // 3
    tris = torch.full((cap, 3, 3), -7.0, dtype=torch.float32, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int32, device="cuda")
    L = m.L
    assert L.extract_mesh(m.h, ctypes.c_void_p(tris.data_ptr()), cap, ctypes.c_void_p(cnt.data_ptr()), None) == 0
    torch.cuda.synchronize()
    assert int(cnt.item()) == len(full)                          # the total, beyond the capacity
    part = tris.cpu().numpy()
    assert np.array_equal(part, full[:cap])                      # the first cap triangles, in order
    assert L.extract_mesh(m.h, None, 10, ctypes.c_void_p(cnt.data_ptr()), None) != 0   # NULL triangles, cap > 0
