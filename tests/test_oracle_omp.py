"""The oracle's OpenMP build (timed as the all-cores CPU baseline) computes
exactly what the single-thread build computes: its parallel loops only
evaluate independent pixels, rows and blocks, and every sum and insertion
is taken in the serial order (no GPU)."""
import numpy as np

import oracle as O
import synth


def run(lib, seq, frames):
    a = O.OracleMap(seq.voxel_size, seq.truncation, seq.depth_max, 255, seq.carve_stride, real_bits=64, lib=lib)
    b = O.OracleMap(seq.voxel_size, seq.truncation, seq.depth_max, 255, seq.carve_stride, real_bits=32, lib=lib)
    T = seq.poses[0]
    poses, masks, ne = [], [], []
    for k in frames:
        fr = O.Frame(seq.depth[k], seq.rgb[k], *seq.intrinsics, depth_scale=seq.depth_scale)
        if k > 0:
            ne.append(a.normal_equations(fr, T, 0, 0.025))
            ne.append(b.mask(fr, T, 0.5, 0.007)["residual"])
        T, mask = O.process_frame(a, fr, T, k, seq.levels, seq.iters, mask_map=b)
        poses.append(T.copy())
        masks.append(None if mask is None else mask.copy())
    return poses, masks, ne, a.export(), b.export()


def test_openmp_build_equals_serial_build():
    seq = synth.dynamic_room(n_frames=4, width=160, height=120, n_clusters=2, movers="in_view")
    omp = O.load_variant("omp")
    omp.orc_set_threads(4)
    assert omp.orc_get_threads() == 4
    ser = run(O.load_variant("serial"), seq, range(4))
    par = run(omp, seq, range(4))
    for x, y in zip(ser[0], par[0]):
        assert np.array_equal(x, y)
    for x, y in zip(ser[1][1:], par[1][1:]):
        assert np.array_equal(x, y)
    for x, y in zip(ser[2], par[2]):
        assert np.array_equal(x, y)
    for ea, eb in ((ser[3], par[3]), (ser[4], par[4])):
        for x, y in zip(ea, eb):
            assert np.array_equal(x, y)
