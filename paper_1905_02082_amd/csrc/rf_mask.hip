// Residual-based dynamics mask (Sec. III-C, Algorithm 1) for gfx950.
//
//   residual_kernel   r = S(T x)^2 per valid pixel, raw = r > gamma tau^2
//                     (with the tracking kernels: its corner blocks resolve
//                     through the tracking tile cache)
//   pixel_pass 0      3x3 erosion (outside the image counts as 0) -> seeds
//   flood_tiles       every 32x32 tile (plus 1-pixel halo) in LDS grows the
//                     seeds to its local fixpoint; a tile whose new border
//                     pixels can reach an unset pixel of a neighbouring tile
//                     marks that tile dirty; a few more parallel passes
//                     re-run only the dirty tiles (most marks made while
//                     neighbours grew concurrently resolve here)
//   flood_finish      one workgroup re-runs dirty tiles, four at a time, until
//                     no tile is dirty: growth is monotone, so the result is
//                     the unique least fixpoint the queue of Algorithm 1
//                     reaches, with no grid-wide barrier
//   pixel_pass 1      3x3 dilation -> final mask
// All passes take a batch of jobs (one map + frame each); the flood-fill
// finish runs one workgroup per job.
// The flood-fill rule: a neighbour n (8-neighbourhood) of a member p joins
// when |D(p) - D(n)| < theta D(p); invalid pixels carry D = 0 and so never
// join nor propagate.
#include "rf_device.h"
#include "rf_internal.h"

namespace rf {

// Per-pixel passes over the batch: 0 erode raw -> seeds, 1 dilate seeds ->
// mask, 2 copy seeds to the caller's eroded output, 3 copy the fill.
__global__ __launch_bounds__(256) void pixel_pass_kernel(Batch b, int pass) {
  const int jb = batch_job(b, blockIdx.x);
  const Job& J = b.job[jb];
  const int W = J.f.W, H = J.f.H;
  const int idx = (blockIdx.x - b.base[jb]) * blockDim.x + threadIdx.x;
  if (idx >= W * H) return;
  if (pass >= 2) {
    uint8_t* dst = (pass == 2) ? J.eroded : J.filled;
    if (dst) dst[idx] = J.m.md[idx];
    return;
  }
  const uint8_t* in = (pass == 0) ? (J.raw ? J.raw : J.mask_out) : J.m.md;
  uint8_t* out = (pass == 0) ? J.m.md : J.mask_out;
  const int u = idx % W, v = idx / W;
  int all = 1, any = 0;
#pragma unroll
  for (int dv = -1; dv <= 1; ++dv)
#pragma unroll
    for (int du = -1; du <= 1; ++du) {
      const int nu = u + du, nv = v + dv;
      const int val = (nu >= 0 && nv >= 0 && nu < W && nv < H) ? (in[nv * W + nu] != 0) : 0;
      all &= val;
      any |= val;
    }
  out[idx] = (uint8_t)(pass == 0 ? all : any);
}

template <int DF>
__device__ __forceinline__ float flood_depth(const FrameDev& f, float dmax, int u, int v) {
  if (u < 0 || v < 0 || u >= f.W || v >= f.H) return 0.0f;
  const float D = load_depth<DF>(f, v * f.W + u);
  return depth_ok(D, dmax) ? D : 0.0f;
}

constexpr int kHalo = kTile + 2;
constexpr int kFloodPasses = 5;  // parallel passes over dirty tiles before the one-workgroup drain

// Grows the seeds of tile (tx,ty) to the tile-local fixpoint.  The halo is
// read-only input.  Marks the neighbouring tiles that a newly set border
// pixel can reach.  The workgroup may hold several groups of nthr threads
// (tid: index in the group), each on a tile of its own with its own LDS
// buffers and flag, all passing the same barriers; a group with active =
// false takes part in the barriers only.  Two groups may hold neighbouring
// tiles: each writes only its own tile's pixels, and a new member on a border
// marks the neighbour, which the caller then runs again, so the result is the
// same least fixpoint.
template <int DF>
__device__ void flood_one_tile(const MapDev& m, const FrameDev& f, float theta, int tx, int ty, bool active,
                               int tiles_x, int tiles_y, uint8_t* s_m, uint8_t* s_m0, float* s_d, int* s_flag,
                               int* s_any, uint32_t* mark, int tid, int nthr) {
  const int u0 = tx * kTile - 1, v0 = ty * kTile - 1;
  if (active) {
    for (int i = tid; i < kHalo * kHalo; i += nthr) {
      const int hu = i % kHalo, hv = i / kHalo;
      const int u = u0 + hu, v = v0 + hv;
      const bool in = (u >= 0 && v >= 0 && u < f.W && v < f.H);
      const uint8_t mv = in ? (m.md[v * f.W + u] != 0) : 0;
      s_m[i] = mv;
      s_m0[i] = mv;
      s_d[i] = flood_depth<DF>(f, m.dmax, u, v);
    }
  }
  __syncthreads();
  // Local fixpoint.  A parallel pass over all pixels (every non-member checks
  // its 8 neighbours) doubles as the convergence test; while it still finds
  // new members, four directional sweeps run (left to right, right to left,
  // top to bottom, bottom to top): lane t walks line t and each step checks
  // the three neighbours on the side already swept, so one sweep carries a
  // path that is monotone in its direction across the tile.
  for (;;) {
    if (tid == 0) *s_flag = 0;
    if (threadIdx.x == 0) *s_any = 0;
    __syncthreads();
    int changed = 0;
    for (int i = tid; active && i < kTile * kTile; i += nthr) {
      const int hu = 1 + (i % kTile), hv = 1 + (i / kTile);
      const int c = hv * kHalo + hu;
      if (s_m[c]) continue;
      const float dq = s_d[c];
      if (!(dq > 0.0f)) continue;
      bool join = false;
#pragma unroll
      for (int dv = -1; dv <= 1; ++dv)
#pragma unroll
        for (int du = -1; du <= 1; ++du) {
          if (!du && !dv) continue;
          const int n = c + dv * kHalo + du;
          if (s_m[n]) {
            const float dp = s_d[n];
            join |= fabsf(dp - dq) < theta * dp;
          }
        }
      if (join) {
        s_m[c] = 1;
        changed = 1;
      }
    }
    if (changed) {
      *s_flag = 1;
      *s_any = 1;
    }
    __syncthreads();
    const int again = *s_flag, any = *s_any;
    __syncthreads();
    if (!any) break;
    // Wavefront w (0..3) sweeps direction w; lane t walks line t.  The three
    // neighbours on the swept side are the lane's own previous cell and its
    // two neighbouring lanes' previous cells, taken from registers by
    // shuffles (the halo lines from LDS), so a step costs no LDS round trip.
    // The four sweeps run concurrently: growth is monotone and the check
    // above runs again after them, so the fixpoint is the same.
    const int t = tid & 63;
    for (int w = tid >> 6; again && w < 4 && t < kTile; w += (nthr >> 6)) {
      const int along = (w < 2) ? 1 : kHalo;   // next cell along the line
      const int across = (w < 2) ? kHalo : 1;  // next line
      const int sgn = (w & 1) ? -1 : 1;
      int c = (1 + t) * across + (1 + ((w & 1) ? kTile - 1 : 0)) * along;
      int cp = c - sgn * along;  // previous cell: the halo
      uint32_t pm = s_m[cp];
      float pd = s_d[cp];
#pragma unroll 1
      for (int i = 0; i < kTile; ++i) {
        uint32_t cm = s_m[c];
        const float cd = s_d[c];
        uint32_t um = (uint32_t)__shfl((int)pm, t > 0 ? t - 1 : 0, 64);
        float ud = __shfl(pd, t > 0 ? t - 1 : 0, 64);
        uint32_t dm = (uint32_t)__shfl((int)pm, t < kTile - 1 ? t + 1 : t, 64);
        float dd = __shfl(pd, t < kTile - 1 ? t + 1 : t, 64);
        if (t == 0) {
          um = s_m[cp - across];
          ud = s_d[cp - across];
        }
        if (t == kTile - 1) {
          dm = s_m[cp + across];
          dd = s_d[cp + across];
        }
        if (!cm && cd > 0.0f) {
          const bool join = (pm && fabsf(pd - cd) < theta * pd) || (um && fabsf(ud - cd) < theta * ud) ||
                            (dm && fabsf(dd - cd) < theta * dd);
          if (join) {
            s_m[c] = 1;
            cm = 1;
          }
        }
        pm = cm;
        pd = cd;
        cp = c;
        c += sgn * along;
      }
    }
    __syncthreads();
  }
  // write back new members; mark neighbours a new border member can reach
  for (int i = tid; active && i < kTile * kTile; i += nthr) {
    const int lu = i % kTile, lv = i / kTile;
    const int c = (lv + 1) * kHalo + (lu + 1);
    if (!s_m[c] || s_m0[c]) continue;
    const int u = u0 + 1 + lu, v = v0 + 1 + lv;
    if (u >= f.W || v >= f.H) continue;
    m.md[v * f.W + u] = 1;
    if (lu != 0 && lu != kTile - 1 && lv != 0 && lv != kTile - 1) continue;
    const float dp = s_d[c];
    for (int dv = -1; dv <= 1; ++dv)
      for (int du = -1; du <= 1; ++du) {
        const int nlu = lu + du, nlv = lv + dv;
        if (nlu >= 0 && nlu < kTile && nlv >= 0 && nlv < kTile) continue;  // inside this tile
        const int n = (nlv + 1) * kHalo + (nlu + 1);
        if (s_m[n]) continue;
        const float dn = s_d[n];
        if (!(dn > 0.0f) || !(fabsf(dp - dn) < theta * dp)) continue;
        const int ntx = tx + (nlu < 0 ? -1 : (nlu >= kTile ? 1 : 0));
        const int nty = ty + (nlv < 0 ? -1 : (nlv >= kTile ? 1 : 0));
        if (ntx < 0 || nty < 0 || ntx >= tiles_x || nty >= tiles_y) continue;
        mark[nty * tiles_x + ntx] = 1;
      }
  }
  __syncthreads();
}

// Parallel pass over the tiles of every job.  Pass 0 takes every tile with a
// member in its halo and marks into dirty buffer 0; pass k > 0 takes the
// tiles marked in buffer (k-1) % 2 (clearing their own flag) and marks into
// buffer k % 2, so no pass reads the flags it writes.
template <int DF>
__global__ __launch_bounds__(256) void flood_tiles_kernel(Batch b, float theta, int pass) {
  __shared__ uint8_t s_m[kHalo * kHalo], s_m0[kHalo * kHalo];
  __shared__ float s_d[kHalo * kHalo];
  __shared__ int s_flag, s_any;
  const int jb = batch_job(b, blockIdx.x);
  const Job& J = b.job[jb];
  const MapDev& m = J.m;
  const FrameDev& f = J.f;
  const int g = blockIdx.x - b.base[jb];
  const int tx = g % J.tiles_x, ty = g / J.tiles_x;
  uint32_t* mark = m.dirty + (size_t)(pass & 1) * m.dirty_cap;
  if (pass > 0) {
    uint32_t* own = m.dirty + (size_t)((pass - 1) & 1) * m.dirty_cap + g;
    if (!*own) return;  // uniform
    __syncthreads();
    if (threadIdx.x == 0) *own = 0;
  } else {
    // skip tiles whose halo holds no member at all
    const int u0 = tx * kTile - 1, v0 = ty * kTile - 1;
    int any = 0;
    for (int i = threadIdx.x; i < kHalo * kHalo; i += blockDim.x) {
      const int u = u0 + i % kHalo, v = v0 + i / kHalo;
      if (u >= 0 && v >= 0 && u < f.W && v < f.H) any |= m.md[v * f.W + u];
    }
    if (!__syncthreads_or(any)) return;
  }
  flood_one_tile<DF>(m, f, theta, tx, ty, true, J.tiles_x, J.tiles_y, s_m, s_m0, s_d, &s_flag, &s_any, mark,
                     threadIdx.x, blockDim.x);
}

// One workgroup per job: process dirty tiles until none is left (or the
// work cap), kFinishGroups tiles at a time (groups of kFinishThreads threads;
// 4 measured faster than 8 or 16 smaller groups).
constexpr int kFinishGroups = 4;
constexpr int kFinishThreads = 1024 / kFinishGroups;
template <int DF>
__global__ __launch_bounds__(1024) void flood_finish_kernel(Batch b, float theta, int buf) {
  __shared__ uint8_t s_m[kFinishGroups][kHalo * kHalo], s_m0[kFinishGroups][kHalo * kHalo];
  __shared__ float s_d[kFinishGroups][kHalo * kHalo];
  __shared__ int s_flag[kFinishGroups], s_any;
  __shared__ int s_list[1024];
  __shared__ int s_n;
  const Job& J = b.job[blockIdx.x];
  const MapDev& m = J.m;
  const FrameDev& f = J.f;
  const int tiles_x = J.tiles_x, tiles_y = J.tiles_y;
  const int ntiles = tiles_x * tiles_y;
  const int max_tiles_processed = 64 * ntiles + f.W * f.H;
  uint32_t* dirty = m.dirty + (size_t)buf * m.dirty_cap;
  int processed = 0;
  for (;;) {
    if (threadIdx.x == 0) s_n = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < ntiles; i += blockDim.x) {
      if (dirty[i]) {
        dirty[i] = 0;
        const int k = atomicAdd(&s_n, 1);
        if (k < 1024) s_list[k] = i;
        else dirty[i] = 1;  // no room this sweep: keep it for the next
      }
    }
    __syncthreads();
    const int n = min(s_n, 1024);
    __syncthreads();
    if (n == 0) break;
    const int q = threadIdx.x / kFinishThreads;  // group
    for (int k = 0; k < n; k += kFinishGroups) {
      const bool act = k + q < n;
      const int tile = act ? s_list[k + q] : 0;
      flood_one_tile<DF>(m, f, theta, tile % tiles_x, tile / tiles_x, act, tiles_x, tiles_y, s_m[q], s_m0[q],
                         s_d[q], &s_flag[q], &s_any, dirty, threadIdx.x % kFinishThreads, kFinishThreads);
    }
    processed += n;
    if (processed > max_tiles_processed) {
      if (threadIdx.x == 0) atomicOr(&m.st->flags, (uint32_t)RF_FLAG_MASK_LIMIT);
      __syncthreads();
      for (int i = threadIdx.x; i < ntiles; i += blockDim.x) dirty[i] = 0;  // leave no flag behind
      break;
    }
  }
}

static int set_bases(Batch& b, int (*count)(const Job&)) {
  int total = 0;
  for (int j = 0; j < b.n; ++j) {
    b.base[j] = total;
    total += count(b.job[j]);
  }
  b.base[b.n] = total;
  return total;
}

static int pixel_groups(const Job& J) { return (J.f.W * J.f.H + 255) / 256; }
static int tile_count(const Job& J) { return J.tiles_x * J.tiles_y; }

template <int DF, int STORAGE>
static void mask_impl(Batch& b, const rf_mask_params& mp, hipStream_t s) {
  bool eroded = false, filled = false;
  for (int j = 0; j < b.n; ++j) {
    Job& J = b.job[j];
    J.tiles_x = (J.f.W + kTile - 1) / kTile;
    J.tiles_y = (J.f.H + kTile - 1) / kTile;
    eroded |= J.eroded != nullptr;
    filled |= J.filled != nullptr;
  }
  launch_residual(b, DF, STORAGE, mp.gamma, s);
  int g = set_bases(b, pixel_groups);
  pixel_pass_kernel<<<g, 256, 0, s>>>(b, 0);
  if (eroded) pixel_pass_kernel<<<g, 256, 0, s>>>(b, 2);
  // the tile flags are all zero here: map initialisation zeroes them, and
  // every mask computation ends with both buffers empty (each parallel pass
  // clears the flags it consumes, the finish drains the last buffer)
  g = set_bases(b, tile_count);
  for (int pass = 0; pass <= kFloodPasses; ++pass) flood_tiles_kernel<DF><<<g, 256, 0, s>>>(b, mp.theta, pass);
  flood_finish_kernel<DF><<<b.n, 1024, 0, s>>>(b, mp.theta, kFloodPasses & 1);
  g = set_bases(b, pixel_groups);
  if (filled) pixel_pass_kernel<<<g, 256, 0, s>>>(b, 3);
  pixel_pass_kernel<<<g, 256, 0, s>>>(b, 1);
}

void launch_mask(Batch& b, int df, int st, const rf_mask_params& mp, hipStream_t s) {
  if (df == RF_DEPTH_U16) {
    if (st == RF_STORAGE_FP32) mask_impl<RF_DEPTH_U16, RF_STORAGE_FP32>(b, mp, s);
    else mask_impl<RF_DEPTH_U16, RF_STORAGE_FP16_U8>(b, mp, s);
  } else {
    if (st == RF_STORAGE_FP32) mask_impl<RF_DEPTH_F32, RF_STORAGE_FP32>(b, mp, s);
    else mask_impl<RF_DEPTH_F32, RF_STORAGE_FP16_U8>(b, mp, s);
  }
}

}  // namespace rf
