"""The C-ABI boundary on the host (no GPU): the built library loads, exports
every symbol include/refusion.h declares, the ctypes layouts match the C
structs, and host-side argument checks report errors without touching the
device."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "refusion.h")


@pytest.fixture(scope="module")
def N():
    from paper_1905_02082_amd import _native
    if not os.path.exists(_native.LIB_PATH):
        pytest.fail("librefusion_hip.so is not built; run __graft_entry__.build()")
    _native.load()
    return _native


def declared_functions():
    src = open(HEADER).read()
    return re.findall(r"^(?:rf_status|const char\*)\s+(\w+)\(", src, re.M)


def test_library_exports_every_declared_symbol(N):
    lib = ctypes.CDLL(N.LIB_PATH)
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(N.EXPORTS), "binding and header disagree"


def test_ctypes_layouts_match_c_header(tmp_path, N):
    prog = tmp_path / "layout.c"
    prog.write_text('''
#include <stdio.h>
#include <stddef.h>
#include "refusion.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu\\n", sizeof(rf_frame), sizeof(rf_map_params), sizeof(rf_track_params),
         sizeof(rf_mask_params), sizeof(rf_track_stats));
  printf("%zu %zu %zu %zu\\n", offsetof(rf_frame, depth), offsetof(rf_frame, rgb),
         offsetof(rf_track_params, lm_lambda), offsetof(rf_track_stats, level_count));
  printf("%zu %zu %zu\\n", sizeof(rf_job), offsetof(rf_job, frame), offsetof(rf_job, d_stats));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(prog), "-o", str(exe)])
    out = subprocess.check_output([str(exe)]).decode().split()
    sizes = [int(x) for x in out[:5]]
    offs = [int(x) for x in out[5:9]]
    job = [int(x) for x in out[9:]]
    assert job == [ctypes.sizeof(N.RfJob), N.RfJob.frame.offset, N.RfJob.d_stats.offset]
    assert sizes == [ctypes.sizeof(N.RfFrame), ctypes.sizeof(N.RfMapParams), ctypes.sizeof(N.RfTrackParams),
                     ctypes.sizeof(N.RfMaskParams), ctypes.sizeof(N.RfTrackStats)]
    assert offs == [N.RfFrame.depth.offset, N.RfFrame.rgb.offset, N.RfTrackParams.lm_lambda.offset,
                    N.RfTrackStats.level_count.offset]


def params(N, **kw):
    d = dict(voxel_size=0.01, truncation=0.03, depth_max=5.0, num_buckets=1 << 20, max_blocks=1 << 17,
             max_weight=255, carve_stride=4, storage=0, max_pixels=640 * 480)
    d.update(kw)
    return N.RfMapParams(**d)


def test_hashmap_bytes_layout(N):
    L = N.load()
    n = ctypes.c_size_t(0)
    p = params(N)
    assert L.hashmap_bytes(ctypes.byref(p), ctypes.byref(n)) == 0
    nb, mb = 1 << 20, 1 << 17
    tcache = (64 + 128 + 512 + 512) * ((640 * 480 + 255) // 256 + 64) * 16   # tracking block cache: pairs per tile at levels 0-3
    tcache += 4 * ((640 * 480 + 255) // 256 + 64) * 4                 # and their counts
    core = nb * 16 + nb + mb * 8 + nb * 4 + mb * 512 * 8 + mb * 512 * 4 + tcache   # buckets + touched-bucket map
    assert core <= n.value <= core + 256 * 16 + 512 * 32 * 8 + 640 * 480 * 2
    p16 = params(N, storage=1)
    n16 = ctypes.c_size_t(0)
    assert L.hashmap_bytes(ctypes.byref(p16), ctypes.byref(n16)) == 0
    assert n.value - n16.value == mb * 512 * 4     # 4 fewer bytes per voxel


@pytest.mark.parametrize("bad", [dict(num_buckets=1000), dict(voxel_size=0.0), dict(max_weight=0),
                                 dict(max_weight=256), dict(carve_stride=0), dict(storage=7),
                                 dict(max_blocks=0), dict(truncation=-1.0)])
def test_invalid_params_rejected_on_host(N, bad):
    L = N.load()
    n = ctypes.c_size_t(0)
    p = params(N, **bad)
    assert L.hashmap_bytes(ctypes.byref(p), ctypes.byref(n)) == N.RF_EINVAL
    assert L.rf_last_error().decode()


def test_create_rejects_small_or_misaligned_arena(N):
    L = N.load()
    p = params(N)
    h = ctypes.c_void_p(0)
    # no device memory is touched: the checks fail before any launch
    assert L.hashmap_create(ctypes.byref(p), ctypes.c_void_p(256), 1024, None, ctypes.byref(h)) == N.RF_ENOMEM
    assert L.hashmap_create(ctypes.byref(p), ctypes.c_void_p(100), 1 << 40, None, ctypes.byref(h)) == N.RF_EINVAL
    assert L.hashmap_create(None, ctypes.c_void_p(256), 1 << 40, None, ctypes.byref(h)) == N.RF_EINVAL


def test_null_handles_rejected(N):
    L = N.load()
    assert L.hashmap_allocate(None, None, None, None, None) == N.RF_EINVAL
    assert L.integrate_frame(None, None, None, None, None) == N.RF_EINVAL
    assert L.track_frame(None, None, None, None, None, None, None) == N.RF_EINVAL
    assert L.compute_dynamic_mask(None, None, None, None, None, None, None) == N.RF_EINVAL
    assert L.map_status(None, None, None, None) == N.RF_EINVAL
    assert L.extract_mesh(None, None, 0, None, None) == N.RF_EINVAL
    assert L.raycast_depth(None, None, None, 0.3, 5.0, 5.0, 1, None, None) == N.RF_EINVAL


def test_raycast_and_mesh_argument_checks(N):
    """Bad ray-cast ranges and a NULL triangle buffer with a capacity are
    rejected on the host, before anything is enqueued (the map handle is a
    dummy pointer that is never dereferenced by these checks)."""
    L = N.load()
    fake = ctypes.c_void_p(0x1000)
    fr = N.RfFrame(100.0, 100.0, 40.0, 30.0, 80, 60, 0x2000, N.RF_DEPTH_F32, 1.0, 0x3000)
    pose, out = ctypes.c_void_p(0x4000), ctypes.c_void_p(0x5000)
    for zn, zf, far, only in [(0.0, 5.0, 5.0, 1), (0.5, 0.4, 5.0, 1), (0.3, 5.0, -1.0, 1), (0.3, 5.0, 5.0, 2)]:
        assert L.raycast_depth(fake, ctypes.byref(fr), pose, zn, zf, far, only, out, None) == N.RF_EINVAL
        assert L.rf_last_error().decode()
    assert L.extract_mesh(fake, None, 10, ctypes.c_void_p(0x6000), None) == N.RF_EINVAL


def test_frame_shape_checks(N):
    """Frames beyond 2^26 pixels, or beyond 2^18 tracking tiles of 16x16
    (the range the fixed-point normal-equation totals are sized for), are
    rejected on the host before the map is used (dummy pointers again)."""
    L = N.load()
    fake = ctypes.c_void_p(0x1000)
    pose, out = ctypes.c_void_p(0x4000), ctypes.c_void_p(0x5000)
    for w, h in [(0, 60), (80, -1), (1 << 14, 1 << 13), (1, 1 << 23), (17, (1 << 26) // 17)]:
        fr = N.RfFrame(100.0, 100.0, 40.0, 30.0, w, h, 0x2000, N.RF_DEPTH_F32, 1.0, 0x3000)
        assert L.raycast_depth(fake, ctypes.byref(fr), pose, 0.3, 5.0, 5.0, 1, out, None) == N.RF_EINVAL, (w, h)
        assert "frame size" in L.rf_last_error().decode()


def test_package_has_no_cpu_fallback():
    """The product package must not import the oracle."""
    pkg = os.path.join(ROOT, "paper_1905_02082_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "liboracle" not in text, f
