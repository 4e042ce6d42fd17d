// extern "C" entry points declared in include/refusion.h: argument checks,
// arena layout and launch orchestration.  No call allocates device memory;
// every buffer comes from the caller (the map arena included).
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "rf_device.h"
#include "rf_internal.h"

struct rf_map {
  rf::HostMap h;
};

namespace {

thread_local char g_err[512] = "";

rf_status fail(rf_status code, const char* fmt, ...) {
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(g_err, sizeof(g_err), fmt, ap);
  va_end(ap);
  return code;
}

rf_status check_launch(const char* what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(RF_EDEVICE, "%s: %s", what, hipGetErrorString(e));
  return RF_OK;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
  size_t st, buckets, block_keys, flist, sdfw, rgb, partials, md, counts, dirty, tcache, tc_count, mesh, cells, wlist,
      touched, total;
  uint32_t dirty_cap, tc_tiles, cells_cap;
};

bool is_pow2(uint32_t x) { return x && !(x & (x - 1)); }

rf_status validate_params(const rf_map_params* p) {
  if (!p) return fail(RF_EINVAL, "params is NULL");
  if (!(p->voxel_size > 0.0f) || !(p->truncation > 0.0f) || !(p->depth_max > 0.0f))
    return fail(RF_EINVAL, "voxel_size, truncation and depth_max must be > 0");
  if (!is_pow2(p->num_buckets) || p->num_buckets < 64) return fail(RF_EINVAL, "num_buckets must be a power of two >= 64");
  if (p->max_blocks == 0 || p->max_blocks >= 0x7FFFFFFFu / 512u)
    return fail(RF_EINVAL, "max_blocks must be in [1, 2^22)");
  if (p->max_weight < 1 || p->max_weight > 255) return fail(RF_EINVAL, "max_weight must be in [1, 255]");
  if (p->carve_stride < 1) return fail(RF_EINVAL, "carve_stride must be >= 1");
  if (p->storage != RF_STORAGE_FP32 && p->storage != RF_STORAGE_FP16_U8) return fail(RF_EINVAL, "unknown storage");
  if (p->max_pixels > (1u << 26)) return fail(RF_EINVAL, "max_pixels too large");
  if (p->free_blocks != 0 && p->free_blocks != 1) return fail(RF_EINVAL, "free_blocks must be 0 or 1");
  if (p->free_blocks && p->num_buckets > (1u << 22))
    return fail(RF_EINVAL, "compact free space needs num_buckets <= 2^22");
  return RF_OK;
}

Layout layout_of(const rf_map_params* p) {
  Layout L;
  size_t o = 0;
  L.st = o; o = align256(o + sizeof(rf::DevState));
  L.buckets = o; o = align256(o + (size_t)p->num_buckets * sizeof(rf::Bucket));
  // buckets touched by an allocation, one byte each, right after the buckets
  // (the kernels find it there)
  L.touched = o; o = align256(o + (size_t)p->num_buckets);
  L.block_keys = o; o = align256(o + (size_t)p->max_blocks * 8);
  L.flist = o; o = align256(o + (size_t)p->num_buckets * 4);
  const size_t rec = (p->storage == RF_STORAGE_FP32) ? 8 : 4;
  L.sdfw = o; o = align256(o + (size_t)p->max_blocks * 512 * rec);
  L.rgb = o; o = align256(o + (size_t)p->max_blocks * 512 * 4);
  L.partials = o; o = align256(o + (size_t)rf::kTrackScratchWords * 8);
  L.md = o; o = align256(o + (size_t)p->max_pixels);
  L.counts = o; o = align256(o + (size_t)rf::kIntegGroups * 16);
  L.dirty_cap = p->max_pixels / 16 + 64;
  L.dirty = o; o = align256(o + (size_t)L.dirty_cap * 2 * 4);  // two flag buffers
  // tracking block cache: the 16x16 tiles of a max_pixels frame plus slack
  // for ragged edges; tiles beyond it use the hash table alone
  L.tc_tiles = (p->max_pixels + 255) / 256 + 64;
  L.tcache = o; o = align256(o + (size_t)rf::tile_refs_before(rf::kCacheLevels) * L.tc_tiles * sizeof(rf::BlockRef));
  L.tc_count = o; o = align256(o + (size_t)rf::kCacheLevels * L.tc_tiles * 4);
  L.mesh = o; o = align256(o + (size_t)2 * rf::kMeshScratch * 4);
  // compact free space: the 8x8 depth cells of a frame of up to max_pixels
  // pixels; ceil(W/8) ceil(H/8) <= W H / 64 + (W + H) / 8 + 1
  L.cells_cap = p->free_blocks ? p->max_pixels / 64 + (p->max_pixels + 1) / 8 + 2 : 0;
  L.cells = o; o = align256(o + (size_t)L.cells_cap * 4);
  // compact free space: the integration's work list (one entry per bucket at most)
  L.wlist = o; o = align256(o + (p->free_blocks ? (size_t)p->num_buckets * 4 : 0));
  L.total = o;
  return L;
}

rf_status make_frame(const rf_frame* f, rf::FrameDev& out) {
  if (!f) return fail(RF_EINVAL, "frame is NULL");
  if (f->width <= 0 || f->height <= 0 || (int64_t)f->width * f->height > (1 << 26) ||
      (int64_t)((f->width + 15) / 16) * ((f->height + 15) / 16) > (1 << 18))  // tracking tiles (fixed-point range)
    return fail(RF_EINVAL, "bad frame size %dx%d", f->width, f->height);
  if (!f->depth || !f->rgb) return fail(RF_EINVAL, "frame depth/rgb is NULL");
  if (f->depth_format != RF_DEPTH_U16 && f->depth_format != RF_DEPTH_F32) return fail(RF_EINVAL, "bad depth_format");
  if (!(f->fx > 0.0f) || !(f->fy > 0.0f)) return fail(RF_EINVAL, "fx, fy must be > 0");
  if (f->depth_format == RF_DEPTH_U16 && !(f->depth_scale > 0.0f)) return fail(RF_EINVAL, "depth_scale must be > 0");
  out.depth = f->depth;
  out.rgb = f->rgb;
  out.W = f->width;
  out.H = f->height;
  out.fx = f->fx;
  out.fy = f->fy;
  out.cx = f->cx;
  out.cy = f->cy;
  out.ifx = 1.0f / f->fx;
  out.ify = 1.0f / f->fy;
  out.dscale = f->depth_scale;
  return RF_OK;
}

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

rf::Job base_job(rf_map* m, const rf::FrameDev& fd) {
  rf::Job J{};
  J.m = m->h.dev;
  J.f = fd;
  return J;
}

// Validates a job list and runs `launch` on chunks of at most kMaxBatch jobs
// that share depth format and storage (the kernels' template parameters).
template <class Fill, class Launch>
rf_status run_batches(const rf_job* jobs, int32_t n, const char* what, Fill fill, Launch launch) {
  if (n < 0 || (n > 0 && !jobs)) return fail(RF_EINVAL, "%s: bad job list", what);
  for (int32_t i = 0; i < n; ++i) {
    if (!jobs[i].map || !jobs[i].d_pose) return fail(RF_EINVAL, "%s: job %d has no map or pose", what, i);
    rf::FrameDev fd;
    rf_status st = make_frame(&jobs[i].frame, fd);
    if (st) return st;
    for (int32_t k = 0; k < i; ++k)
      if (jobs[k].map == jobs[i].map) return fail(RF_EINVAL, "%s: map of job %d appears twice", what, i);
  }
  // every job is checked before anything is enqueued
  std::vector<rf::Job> prepared(n);
  for (int32_t k = 0; k < n; ++k) {
    rf::FrameDev fd;
    make_frame(&jobs[k].frame, fd);
    prepared[k] = base_job(jobs[k].map, fd);
    rf_status st = fill(jobs[k], prepared[k]);
    if (st) return st;
  }
  std::vector<int> done(n, 0);
  for (int32_t i = 0; i < n; ++i) {
    if (done[i]) continue;
    const int df = jobs[i].frame.depth_format, sto = jobs[i].map->h.p.storage;
    rf::Batch b{};
    b.n = 0;
    for (int32_t k = i; k < n; ++k) {
      if (done[k] || jobs[k].frame.depth_format != df || jobs[k].map->h.p.storage != sto) continue;
      b.job[b.n++] = prepared[k];
      done[k] = 1;
      if (b.n == rf::kMaxBatch) {
        launch(b, df, sto);
        b.n = 0;
      }
    }
    if (b.n) launch(b, df, sto);
  }
  return check_launch(what);
}

rf_status mask_checks(const rf_job& j, rf::Job& J) {
  if (!j.d_mask_out) return fail(RF_EINVAL, "compute_dynamic_mask: mask output is NULL");
  const uint32_t npx = (uint32_t)J.f.W * (uint32_t)J.f.H;
  if (npx > j.map->h.p.max_pixels)
    return fail(RF_ENOMEM, "frame has %u pixels, map max_pixels is %u", npx, j.map->h.p.max_pixels);
  const uint32_t tiles =
      (uint32_t)((J.f.W + rf::kTile - 1) / rf::kTile) * (uint32_t)((J.f.H + rf::kTile - 1) / rf::kTile);
  if (tiles > j.map->h.dev.dirty_cap) return fail(RF_ENOMEM, "flood-fill tile table too small");
  J.pose = j.d_pose;
  J.mask_out = j.d_mask_out;
  return RF_OK;
}

// ------------------------------------------- allocation-free mask variant
// compute_dynamic_mask_static keeps the flood fill's per-pixel mask and its
// two buffers of tile flags in this file-scope device array instead of the
// map arena.  Each GPU holds its own copy at its own address until the
// process ends; host code uses only the address hipGetSymbolAddress returns
// for the current device, never the array's name.
constexpr size_t kStaticScratchBytes = (size_t)4 << 20;
__device__ __align__(256) uint8_t scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device (looked up once per device).
rf_status static_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(RF_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(RF_EUNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return fail(RF_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return RF_OK;
}

__global__ void clear_words_kernel(uint32_t* p, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0u;
}

}  // namespace

extern "C" {

const char* rf_last_error(void) { return g_err; }

const char* rf_version(void) { return "refusion-gfx950 1.0"; }

rf_status hashmap_bytes(const rf_map_params* p, size_t* bytes) {
  rf_status st = validate_params(p);
  if (st) return st;
  if (!bytes) return fail(RF_EINVAL, "bytes is NULL");
  *bytes = layout_of(p).total;
  return RF_OK;
}

rf_status hashmap_create(const rf_map_params* p, void* arena, size_t bytes, void* stream, rf_map** out) {
  rf_status st = validate_params(p);
  if (st) return st;
  if (!arena || !out) return fail(RF_EINVAL, "arena/out is NULL");
  if (reinterpret_cast<uintptr_t>(arena) & 255) return fail(RF_EINVAL, "arena must be 256-byte aligned");
  const Layout L = layout_of(p);
  if (bytes < L.total) return fail(RF_ENOMEM, "arena has %zu bytes, needs %zu", bytes, L.total);
  rf_map* m = new (std::nothrow) rf_map;
  if (!m) return fail(RF_ENOMEM, "host allocation failed");
  char* a = static_cast<char*>(arena);
  rf::HostMap& h = m->h;
  h.p = *p;
  h.arena = arena;
  h.bytes = bytes;
  rf::MapDev& d = h.dev;
  d.st = reinterpret_cast<rf::DevState*>(a + L.st);
  d.buckets = reinterpret_cast<rf::Bucket*>(a + L.buckets);
  d.bucket_mask = p->num_buckets - 1;
  d.max_probe = p->num_buckets < 1024 ? p->num_buckets : 1024;
  d.block_keys = reinterpret_cast<unsigned long long*>(a + L.block_keys);
  d.flist = reinterpret_cast<uint32_t*>(a + L.flist);
  d.flist_cap = p->num_buckets;
  d.max_blocks = p->max_blocks;
  d.sdfw = a + L.sdfw;
  d.rgb = reinterpret_cast<uchar4*>(a + L.rgb);
  d.partials = reinterpret_cast<double*>(a + L.partials);
  d.md = reinterpret_cast<uint8_t*>(a + L.md);
  d.integ_counts = reinterpret_cast<uint4*>(a + L.counts);
  d.cells = reinterpret_cast<float*>(a + L.cells);
  d.cells_cap = L.cells_cap;
  d.free_blocks = p->free_blocks ? 1u : 0u;
  d.wlist = p->free_blocks ? reinterpret_cast<uint32_t*>(a + L.wlist) : nullptr;
  d.dirty = reinterpret_cast<uint32_t*>(a + L.dirty);
  d.tcache = reinterpret_cast<rf::BlockRef*>(a + L.tcache);
  d.tc_count = reinterpret_cast<uint32_t*>(a + L.tc_count);
  d.mesh_scratch = reinterpret_cast<uint32_t*>(a + L.mesh);
  d.tc_tiles = L.tc_tiles;
  d.max_pixels = p->max_pixels;
  d.dirty_cap = L.dirty_cap;
  d.s = p->voxel_size;
  d.is = 1.0f / p->voxel_size;
  d.iB = 1.0f / (8.0f * p->voxel_size);
  d.tau = p->truncation;
  d.inv_tau = 1.0f / p->truncation;
  d.dmax = p->depth_max;
  d.max_weight = (float)p->max_weight;
  d.carve_stride = p->carve_stride;
  rf::launch_map_init(d, p->num_buckets, p->storage, S(stream));
  st = check_launch("hashmap_create");
  if (st) {
    delete m;
    return st;
  }
  *out = m;
  return RF_OK;
}

rf_status hashmap_destroy(rf_map* m) {
  delete m;
  return RF_OK;
}

rf_status hashmap_reset(rf_map* m, void* stream) {
  if (!m) return fail(RF_EINVAL, "map is NULL");
  rf::launch_map_init(m->h.dev, m->h.p.num_buckets, m->h.p.storage, S(stream));
  return check_launch("hashmap_reset");
}

rf_status hashmap_allocate(rf_map* m, const rf_frame* f, const double* d_pose, const uint8_t* d_mask, void* stream) {
  if (!m || !d_pose || !f) return fail(RF_EINVAL, "map/pose/frame is NULL");
  rf_job j{};
  j.map = m;
  j.frame = *f;
  j.d_pose = const_cast<double*>(d_pose);
  j.d_mask = d_mask;
  return hashmap_allocate_batch(&j, 1, stream);
}

rf_status integrate_frame(rf_map* m, const rf_frame* f, const double* d_pose, const uint8_t* d_mask, void* stream) {
  if (!m || !d_pose || !f) return fail(RF_EINVAL, "map/pose/frame is NULL");
  rf_job j{};
  j.map = m;
  j.frame = *f;
  j.d_pose = const_cast<double*>(d_pose);
  j.d_mask = d_mask;
  return integrate_frame_batch(&j, 1, stream);
}

rf_status track_frame(rf_map* m, const rf_frame* f, const rf_track_params* tp, const uint8_t* d_mask,
                      double* d_pose_inout, rf_track_stats* d_stats, void* stream) {
  if (!m || !tp || !d_pose_inout || !f) return fail(RF_EINVAL, "map/params/pose/frame is NULL");
  rf_job j{};
  j.map = m;
  j.frame = *f;
  j.d_pose = d_pose_inout;
  j.d_mask = d_mask;
  j.d_stats = d_stats;
  return track_frame_batch(&j, 1, tp, stream);
}

rf_status track_normal_equations(rf_map* m, const rf_frame* f, const uint8_t* d_mask, const double* d_pose,
                                 int32_t level, float w_c, double* d_out29, void* stream) {
  if (!m || !d_pose || !d_out29) return fail(RF_EINVAL, "map/pose/out is NULL");
  if (level < 0 || level > 7) return fail(RF_EINVAL, "level must be in [0,7]");
  rf::FrameDev fd;
  rf_status st = make_frame(f, fd);
  if (st) return st;
  rf::Batch b{};
  b.n = 1;
  b.job[0] = base_job(m, fd);
  b.job[0].mask = d_mask;
  b.job[0].pose = const_cast<double*>(d_pose);
  rf::launch_normal_equations(b, f->depth_format, m->h.p.storage, level, w_c, d_out29, S(stream));
  return check_launch("track_normal_equations");
}

rf_status compute_dynamic_mask_stages(rf_map* m, const rf_frame* f, const double* d_pose, const rf_mask_params* mp,
                                      uint8_t* d_raw, uint8_t* d_eroded, uint8_t* d_filled, uint8_t* d_mask_out,
                                      float* d_residual_out, void* stream) {
  if (!m || !d_pose || !mp || !d_mask_out || !f) return fail(RF_EINVAL, "map/pose/params/out/frame is NULL");
  if (!(mp->gamma >= 0.0f) || !(mp->theta >= 0.0f)) return fail(RF_EINVAL, "gamma and theta must be >= 0");
  rf_job j{};
  j.map = m;
  j.frame = *f;
  j.d_pose = const_cast<double*>(d_pose);
  j.d_mask_out = d_mask_out;
  rf::FrameDev fd;
  rf_status st = make_frame(f, fd);
  if (st) return st;
  auto fill = [&](const rf_job& jj, rf::Job& J) -> rf_status {
    rf_status s2 = mask_checks(jj, J);
    if (s2) return s2;
    J.raw = d_raw;
    J.eroded = d_eroded;
    J.filled = d_filled;
    J.residual = d_residual_out;
    return RF_OK;
  };
  auto launch = [&](rf::Batch& b, int df, int sto) { rf::launch_mask(b, df, sto, *mp, S(stream)); };
  return run_batches(&j, 1, "compute_dynamic_mask", fill, launch);
}

rf_status compute_dynamic_mask(rf_map* m, const rf_frame* f, const double* d_pose, const rf_mask_params* mp,
                               uint8_t* d_mask_out, float* d_residual_out, void* stream) {
  return compute_dynamic_mask_stages(m, f, d_pose, mp, nullptr, nullptr, nullptr, d_mask_out, d_residual_out, stream);
}

rf_status compute_dynamic_mask_static(rf_map* m, const rf_frame* f, const double* d_pose, const rf_mask_params* mp,
                                      uint8_t* d_mask_out, float* d_residual_out, void* stream) {
  if (!m || !d_pose || !mp || !d_mask_out || !f) return fail(RF_EINVAL, "map/pose/params/out/frame is NULL");
  if (!(mp->gamma >= 0.0f) || !(mp->theta >= 0.0f)) return fail(RF_EINVAL, "gamma and theta must be >= 0");
  rf::FrameDev fd;
  rf_status st = make_frame(f, fd);
  if (st) return st;
  // the flood fill's scratch: the per-pixel mask, then two buffers of tile flags
  const size_t npx = (size_t)fd.W * (size_t)fd.H;
  const uint32_t tiles = (uint32_t)((fd.W + rf::kTile - 1) / rf::kTile) * (uint32_t)((fd.H + rf::kTile - 1) / rf::kTile);
  const size_t flags_at = align256(npx);
  const size_t need = flags_at + (size_t)2 * tiles * 4;
  if (need > kStaticScratchBytes)
    return fail(RF_ENOMEM, "compute_dynamic_mask_static: a %dx%d frame needs %zu bytes of scratch, the static "
                "array holds %zu", fd.W, fd.H, need, kStaticScratchBytes);
  void* base = nullptr;
  st = static_scratch(&base);
  if (st) return st;
  uint8_t* sp = static_cast<uint8_t*>(base);
  rf_job j{};
  j.map = m;
  j.frame = *f;
  j.d_pose = const_cast<double*>(d_pose);
  j.d_mask_out = d_mask_out;
  auto fill = [&](const rf_job& jj, rf::Job& J) -> rf_status {
    if (!jj.d_mask_out) return fail(RF_EINVAL, "compute_dynamic_mask_static: mask output is NULL");
    J.pose = jj.d_pose;
    J.mask_out = jj.d_mask_out;
    J.residual = d_residual_out;
    J.m.md = sp;
    J.m.dirty = reinterpret_cast<uint32_t*>(sp + flags_at);
    J.m.dirty_cap = tiles;
    return RF_OK;
  };
  auto launch = [&](rf::Batch& b, int df, int sto) {
    // the tile flags must start empty; the last call on this device may
    // have used other sizes (a fill kernel, no memset node in a captured graph)
    clear_words_kernel<<<(2 * tiles + 255) / 256, 256, 0, S(stream)>>>(b.job[0].m.dirty, 2 * tiles);
    rf::launch_mask(b, df, sto, *mp, S(stream));
  };
  return run_batches(&j, 1, "compute_dynamic_mask_static", fill, launch);
}

// ---------------------------------------------------------------- batched entry points
rf_status hashmap_allocate_batch(const rf_job* jobs, int32_t n, void* stream) {
  auto fill = [&](const rf_job& j, rf::Job& J) -> rf_status {
    J.pose = j.d_pose;
    J.mask = j.d_mask;
    return RF_OK;
  };
  auto launch = [&](rf::Batch& b, int df, int) { rf::launch_allocate(b, df, S(stream)); };
  return run_batches(jobs, n, "hashmap_allocate", fill, launch);
}

rf_status integrate_frame_batch(const rf_job* jobs, int32_t n, void* stream) {
  auto fill = [&](const rf_job& j, rf::Job& J) -> rf_status {
    J.pose = j.d_pose;
    J.mask = j.d_mask;
    J.cells_w = J.cells_h = 0;
    if (J.m.free_blocks) {
      // compact free space: the frame's depth cells must fit the map's
      const uint32_t npx = (uint32_t)J.f.W * (uint32_t)J.f.H;
      if (npx > j.map->h.p.max_pixels)
        return fail(RF_ENOMEM, "integrate_frame: frame has %u pixels, map max_pixels is %u", npx,
                    j.map->h.p.max_pixels);
      J.cells_w = (J.f.W + rf::kCell - 1) / rf::kCell;
      J.cells_h = (J.f.H + rf::kCell - 1) / rf::kCell;
    }
    return RF_OK;
  };
  auto launch = [&](rf::Batch& b, int df, int sto) { rf::launch_integrate(b, df, sto, S(stream)); };
  return run_batches(jobs, n, "integrate_frame", fill, launch);
}

rf_status track_frame_batch(const rf_job* jobs, int32_t n, const rf_track_params* tp, void* stream) {
  if (!tp) return fail(RF_EINVAL, "track params are NULL");
  if (tp->levels < 1 || tp->levels > 8 || tp->iters_per_level < 0 || tp->iters_per_level > 1000)
    return fail(RF_EINVAL, "levels must be in [1,8], iters_per_level in [0,1000]");
  if (!(tp->lm_lambda >= 0.0)) return fail(RF_EINVAL, "lm_lambda must be >= 0");
  if (tp->adaptive != 0 && tp->adaptive != 1) return fail(RF_EINVAL, "adaptive must be 0 or 1");
  auto fill = [&](const rf_job& j, rf::Job& J) -> rf_status {
    J.pose = j.d_pose;
    J.mask = j.d_mask;
    J.stats = j.d_stats;
    return RF_OK;
  };
  auto launch = [&](rf::Batch& b, int df, int sto) { rf::launch_track(b, df, sto, *tp, S(stream)); };
  return run_batches(jobs, n, "track_frame", fill, launch);
}

rf_status compute_dynamic_mask_batch(const rf_job* jobs, int32_t n, const rf_mask_params* mp, void* stream) {
  if (!mp) return fail(RF_EINVAL, "mask params are NULL");
  if (!(mp->gamma >= 0.0f) || !(mp->theta >= 0.0f)) return fail(RF_EINVAL, "gamma and theta must be >= 0");
  auto fill = [&](const rf_job& j, rf::Job& J) -> rf_status { return mask_checks(j, J); };
  auto launch = [&](rf::Batch& b, int df, int sto) { rf::launch_mask(b, df, sto, *mp, S(stream)); };
  return run_batches(jobs, n, "compute_dynamic_mask", fill, launch);
}

rf_status extract_surface(rf_map* m, float* d_points, uint32_t cap, uint32_t* d_count, void* stream) {
  if (!m || !d_count || (cap && !d_points)) return fail(RF_EINVAL, "map/count/points is NULL");
  rf::launch_surface(m->h.dev, m->h.p.storage, d_points, cap, d_count, S(stream));
  return check_launch("extract_surface");
}

rf_status raycast_depth(rf_map* m, const rf_frame* f, const double* d_pose, float z_near, float z_far,
                        float far_value, int32_t only_invalid, float* d_out, void* stream) {
  if (!m || !f || !d_pose || !d_out) return fail(RF_EINVAL, "map/frame/pose/out is NULL");
  if (!(z_near > 0.0f) || !(z_far > z_near) || !(far_value >= 0.0f))
    return fail(RF_EINVAL, "need 0 < z_near < z_far and far_value >= 0");
  if (only_invalid != 0 && only_invalid != 1) return fail(RF_EINVAL, "only_invalid must be 0 or 1");
  rf::FrameDev fd;
  rf_status st = make_frame(f, fd);
  if (st) return st;
  rf::launch_raycast(m->h.dev, fd, f->depth_format, m->h.p.storage, d_pose, z_near, z_far, far_value, only_invalid,
                     d_out, S(stream));
  return check_launch("raycast_depth");
}

rf_status extract_mesh(rf_map* m, float* d_tris, uint32_t cap, uint32_t* d_count, void* stream) {
  if (!m || !d_count || (cap && !d_tris)) return fail(RF_EINVAL, "map/count/triangles is NULL");
  rf::launch_mesh(m->h.dev, m->h.p.storage, d_tris, cap, d_count, S(stream));
  return check_launch("extract_mesh");
}

rf_status map_status(rf_map* m, void* stream, uint32_t* flags, uint32_t* n_blocks) {
  if (!m) return fail(RF_EINVAL, "map is NULL");
  rf::DevState hs;
  hipError_t e = hipMemcpyAsync(&hs, m->h.dev.st, sizeof(hs), hipMemcpyDeviceToHost, S(stream));
  if (e == hipSuccess) e = hipStreamSynchronize(S(stream));
  if (e != hipSuccess) return fail(RF_EDEVICE, "map_status: %s", hipGetErrorString(e));
  if (flags) *flags = hs.flags;
  if (n_blocks) *n_blocks = hs.n_blocks < m->h.p.max_blocks ? hs.n_blocks : m->h.p.max_blocks;
  return RF_OK;
}

rf_status hashmap_frame_blocks(rf_map* m, int32_t* d_keys, uint32_t cap, uint32_t* d_count, void* stream) {
  if (!m || !d_count || (cap && !d_keys)) return fail(RF_EINVAL, "map/count/keys is NULL");
  rf::launch_frame_blocks(m->h.dev, d_keys, cap, d_count, S(stream));
  return check_launch("hashmap_frame_blocks");
}

rf_status hashmap_export_free(rf_map* m, int32_t* d_keys, float* d_weight, uint32_t cap, uint32_t* d_count,
                              void* stream) {
  if (!m || !d_count || (cap && !d_keys)) return fail(RF_EINVAL, "map/count/keys is NULL");
  rf::launch_export_free(m->h.dev, m->h.p.num_buckets, d_keys, d_weight, cap, d_count, S(stream));
  return check_launch("hashmap_export_free");
}

rf_status hashmap_export(rf_map* m, int32_t* d_keys, float* d_sdf, float* d_weight, uint8_t* d_rgb, uint32_t cap,
                         uint32_t* d_count, void* stream) {
  if (!m || !d_count) return fail(RF_EINVAL, "map/count is NULL");
  rf::launch_export(m->h.dev, m->h.p.storage, d_keys, d_sdf, d_weight, d_rgb, cap, d_count, S(stream));
  return check_launch("hashmap_export");
}

rf_status hashmap_import(rf_map* m, const int32_t* d_keys, const float* d_sdf, const float* d_weight,
                         const uint8_t* d_rgb, uint32_t n, void* stream) {
  if (!m) return fail(RF_EINVAL, "map is NULL");
  if (n && (!d_keys || !d_sdf || !d_weight || !d_rgb)) return fail(RF_EINVAL, "import arrays are NULL");
  rf::launch_import(m->h.dev, m->h.p.storage, d_keys, d_sdf, d_weight, d_rgb, n, S(stream));
  return check_launch("hashmap_import");
}

}  // extern "C"
