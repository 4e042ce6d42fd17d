// Block allocation (Sec. III-A, III-D) and TSDF integration with free-space
// carving (Sec. III-A, III-C, III-D) for gfx950.
//
// Allocation: one thread per pixel walks the block grid along its band (or
// carve) segment with a DDA; each visited block is inserted into the hash by
// CAS and its bucket marked in a byte map of touched buckets by a plain store
// (every ray that touches it stores the same value, so no exchange is
// needed).  Carve rays run in workgroups of their own; cells are probed 12 at
// a time, with their bucket loads and marks each issued together.  A second
// kernel then lists the marked buckets, clearing the marks: the frame's block
// list, each touched block once.
//
// Integration: workgroups stride over the listed blocks, 256 threads x 2
// voxels per block, two blocks per step, each workgroup's list entries and
// buckets read into LDS up front; only voxels the frame updates are
// written.  Records are SoA per block, so a workgroup's loads and stores are
// contiguous 4-KiB (FP32) / 2-KiB (FP16) runs.
#include <type_traits>

#include "rf_device.h"
#include "rf_internal.h"

namespace rf {

// False when the lane just below holds the same key (and is active with a
// valid cell): of a run of equal keys on consecutive lanes only the first
// probes, inserts and marks.  Neighbouring rays (consecutive pixels or
// carve-grid pixels) mostly visit the same blocks in the same order, so this
// removes most duplicates for a few instructions; duplicates that remain are
// harmless (the CAS insert resolves them, and a mark stored twice is one).
__device__ __forceinline__ bool leads_run(unsigned long long key, bool valid, unsigned long long active) {
  const int lane = threadIdx.x & 63;
  const unsigned long long vmask = __ballot(valid) & active;
  // lane - 1's key, moved by a wavefront shift (DPP) rather than an LDS
  // permute; lane 0 and lanes whose neighbour is not valid ignore it
  const unsigned int klo = __builtin_amdgcn_update_dpp(0u, (unsigned int)key, 0x138, 0xF, 0xF, false);
  const unsigned int khi = __builtin_amdgcn_update_dpp(0u, (unsigned int)(key >> 32), 0x138, 0xF, 0xF, false);
  const bool below_same = lane > 0 && ((vmask >> (lane - 1)) & 1ull) &&
                          ((((unsigned long long)khi << 32) | klo) == key);
  return valid && !below_same;
}

// Block-grid DDA of segment q0 -> q1 (block units): cells c = floor(q0) ...
// e = floor(q1), exactly |e-c|_1 steps, each along the axis with the smallest
// next-boundary parameter among the axes not yet at e (ties: x, y, z).  Cells
// are produced in batches of 12 whose home buckets are loaded together, so a
// ray costs one hash round trip per 12 cells instead of one per cell.
struct Dda {
  int c[3], e[3], step[3];
  float tmax[3], tdel[3];
  int left;  // cells still to emit, the current one included

  __device__ __forceinline__ void init(const float q0[3], const float q1[3]) {
    int n = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      c[a] = (int)floorf(q0[a]);
      e[a] = (int)floorf(q1[a]);
      const float d = q1[a] - q0[a];
      step[a] = (e[a] > c[a]) ? 1 : ((e[a] < c[a]) ? -1 : 0);
      if (step[a] != 0) {
        const float inv = 1.0f / d;
        const float bound = (float)(c[a] + (step[a] > 0 ? 1 : 0));
        tmax[a] = (bound - q0[a]) * inv;
        tdel[a] = (float)step[a] * inv;
      } else {
        tmax[a] = INFINITY;
        tdel[a] = INFINITY;
      }
      n += abs(e[a] - c[a]);
    }
    left = n + 1;
  }
  // Branch-free step: the axis with the smallest next-boundary parameter
  // among those not yet at the end cell, ties to x, then y (the same choice
  // as scanning x, y, z and keeping the first strict minimum).
  __device__ __forceinline__ void advance() {
    const float bx = (c[0] != e[0]) ? tmax[0] : INFINITY;
    const float by = (c[1] != e[1]) ? tmax[1] : INFINITY;
    const float bz = (c[2] != e[2]) ? tmax[2] : INFINITY;
    const bool px = bx <= by && bx <= bz;
    const bool py = !px && by <= bz;
    const bool pz = !px && !py;
    c[0] += px ? step[0] : 0;
    c[1] += py ? step[1] : 0;
    c[2] += pz ? step[2] : 0;
    tmax[0] = px ? tmax[0] + tdel[0] : tmax[0];
    tmax[1] = py ? tmax[1] + tdel[1] : tmax[1];
    tmax[2] = pz ? tmax[2] + tdel[2] : tmax[2];
  }
};

// One thread's ray: its cells' blocks are inserted if absent and their
// buckets marked as touched.
template <int DF>
__device__ __forceinline__ void alloc_ray(const Job& J, int g) {
  const MapDev& m = J.m;
  uint8_t* touched = touched_map(m);
  const FrameDev& f = J.f;
  int u, v;
  const int s_c = (int)m.carve_stride;
  if (g < J.carve_groups) {
    const int j = g * blockDim.x + threadIdx.x;
    if (j >= J.carve_w * J.carve_h) return;
    u = (j % J.carve_w) * s_c;
    v = (j / J.carve_w) * s_c;
  } else {
    const int idx = (g - J.carve_groups) * blockDim.x + threadIdx.x;
    if (idx >= f.W * f.H) return;
    u = idx % f.W;
    v = idx / f.W;
    if (u % s_c == 0 && v % s_c == 0) return;
  }
  const uint8_t* mask = J.mask;
  const double* pose = J.pose;
  const int idx = v * f.W + u;
  const float D = load_depth<DF>(f, idx);
  if (!(D > 0.0f)) return;  // no measurement
  if (mask && mask[idx]) return;
  const bool carve = (u % s_c == 0) && (v % s_c == 0);
  // A measurement beyond depth_max (the clipping plane) is too far to be
  // integrated but still shows free space up to the plane (Sec. III-D): only
  // its carve segment is walked, and it ends at the clipping plane.
  const bool far = !(D <= m.dmax);
  if (far && !carve) return;
  float R[9], t[3];
  load_pose_f(pose, R, t);
  const float zn = carve ? 0.0f : fmaxf(D - m.tau, 0.0f);
  const float zf = far ? m.dmax : D + m.tau;
  const float rx = ((float)u - f.cx) * f.ifx, ry = ((float)v - f.cy) * f.ify;
  const float X0[3] = {rx * zn, ry * zn, zn}, X1[3] = {rx * zf, ry * zf, zf};
  float P0[3], P1[3];
  xform(R, t, X0, P0);
  xform(R, t, X1, P1);
  float q0[3], q1[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    q0[a] = P0[a] * m.iB;
    q1[a] = P1[a] * m.iB;
    if (!(fabsf(q0[a]) < kMaxBlockCoord && fabsf(q1[a]) < kMaxBlockCoord)) return;
  }
  Dda d;
  d.init(q0, q1);
  constexpr int kBatch = 12;
  while (d.left > 0) {
    int cx[kBatch], cy[kBatch], cz[kBatch];
    bool ok[kBatch];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      ok[q] = d.left > 0;
      cx[q] = d.c[0];
      cy[q] = d.c[1];
      cz[q] = d.c[2];
      if (ok[q]) {
        --d.left;
        if (d.left > 0) d.advance();
      }
    }
    unsigned long long key[kBatch], bkey[kBatch];
    uint32_t hb[kBatch];
    const unsigned long long active = __ballot(true);
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      key[q] = pack_key(cx[q], cy[q], cz[q]);
      ok[q] = leads_run(key[q], ok[q], active);
      if (!ok[q]) continue;
      hb[q] = hash3(cx[q], cy[q], cz[q]) & m.bucket_mask;
      bkey[q] = m.buckets[hb[q]].key;
    }
    // Cells whose home bucket holds another block: the keys of the next
    // two buckets, loaded for all of them together (linear probing puts
    // most displaced blocks there), before any probes on.
    unsigned long long k1[kBatch], k2[kBatch];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      k1[q] = k2[q] = kEmptyKey;
      if (ok[q] && bkey[q] != key[q] && bkey[q] != kEmptyKey) {
        k1[q] = m.buckets[(hb[q] + 1u) & m.bucket_mask].key;
        k2[q] = m.buckets[(hb[q] + 2u) & m.bucket_mask].key;
      }
    }
    // Mark every cell's bucket as touched (stores issued together); an absent
    // block is inserted first
    int hq[kBatch];
    bool claimed[kBatch];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      hq[q] = -1;
      claimed[q] = false;
      if (!ok[q]) continue;
      int h = (int)hb[q];
      if (bkey[q] == kEmptyKey) {
        h = find_or_claim_from(m, cx[q], cy[q], cz[q], hb[q], 0u, kEmptyKey, &claimed[q]);
      } else if (bkey[q] != key[q]) {
        if (k1[q] == key[q]) h = (int)((hb[q] + 1u) & m.bucket_mask);
        else if (k2[q] == key[q]) h = (int)((hb[q] + 2u) & m.bucket_mask);
        else {
          // absent (insert at the first empty bucket) or further on
          const uint32_t i0 = (k1[q] == kEmptyKey) ? 1u : 2u;
          const unsigned long long k0 = (i0 == 1u) ? k1[q] : k2[q];
          h = find_or_claim_from(m, cx[q], cy[q], cz[q], hb[q], i0, k0, &claimed[q]);
        }
      }
      hq[q] = h;
      if (h >= 0) touched[h] = 1;
    }
    // The blocks this batch inserted: key counts and pool slots (compact
    // free-space maps: none) with one counter atomic per wavefront and cell.
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      const unsigned long long bal = __ballot(claimed[q]);
      if (bal == 0ull) continue;  // uniform
      const int leader = __ffsll((long long)bal) - 1;
      const uint32_t cnt = (uint32_t)__popcll(bal);
      uint32_t base = 0;
      if (lane == leader) {
        atomicAdd(&m.st->n_keys, cnt);
        if (!m.free_blocks) base = atomicAdd(&m.st->n_blocks, cnt);
      }
      base = __shfl(base, leader);
      if (!claimed[q]) continue;
      uint32_t slot = kFreeSlot;  // a free block: no voxels until one of them gets a band update
      if (!m.free_blocks) {
        slot = base + __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
        if (slot < m.max_blocks) {
          m.block_keys[slot] = key[q];
        } else {
          slot = kInvalidSlot;
          atomicOr(&m.st->flags, (uint32_t)RF_FLAG_POOL_FULL);
        }
      }
      m.buckets[hq[q]].slot = slot;
    }
  }
}

template <int DF>
__global__ __launch_bounds__(256) void alloc_kernel(Batch b) {
  // Per job: workgroups [0, carve_groups) take the carve segments of the
  // carve-grid pixels, the rest the band segments of the other pixels, so the
  // long rays share wavefronts with rays of similar length; the carve
  // workgroups come first so that the longest chains start first.
  const int jb = batch_job(b, blockIdx.x);
  alloc_ray<DF>(b.job[jb], blockIdx.x - b.base[jb]);
}

// The frame's block list: every bucket marked as touched, appended in runs
// gathered per workgroup in LDS (one counter atomic per workgroup and run;
// the order of the list is not fixed, its content is), the marks cleared on
// the way.  One workgroup per CU and job streams a contiguous range of the
// byte map, 16 buckets per load.
constexpr int kListGroups = 256;   // workgroups of the listing (all jobs together)
constexpr uint32_t kListRun = 2048;

__global__ __launch_bounds__(256) void list_frame_kernel(Batch b) {
  __shared__ uint32_t s_run[kListRun];
  __shared__ uint32_t s_n, s_base;
  const int jb = batch_job(b, blockIdx.x);
  const MapDev& m = b.job[jb].m;
  const uint32_t nc = (m.bucket_mask + 16u) / 16u;  // 16-byte chunks of the map
  const uint32_t g0 = blockIdx.x - b.base[jb], gn = b.base[jb + 1] - b.base[jb];
  const uint32_t per = (nc + gn - 1) / gn;
  const uint32_t c0 = g0 * per, c1 = min(c0 + per, nc);
  uint4* map = reinterpret_cast<uint4*>(touched_map(m));
  if (threadIdx.x == 0) s_n = 0;
  __syncthreads();
  for (uint32_t cb = c0; cb < c1; cb += blockDim.x) {  // uniform
    const uint32_t c = cb + threadIdx.x;
    const uint4 w = c < c1 ? map[c] : make_uint4(0u, 0u, 0u, 0u);
    const uint32_t words[4] = {w.x, w.y, w.z, w.w};
    uint32_t cnt = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) cnt += __popc(words[k] & 0x01010101u);
    if (cnt) map[c] = make_uint4(0u, 0u, 0u, 0u);
    // positions in the workgroup's run: a prefix over the wavefront's counts
    // (shuffles), one LDS atomic per wavefront
    uint32_t pre = cnt;
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t t = __shfl_up(pre, o);
      if (lane >= o) pre += t;
    }
    const uint32_t total = __shfl(pre, 63);
    uint32_t base = 0;
    if (total && lane == 63) base = atomicAdd(&s_n, total);  // LDS
    base = __shfl(base, 63);
    uint32_t i = base + pre - cnt;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
#pragma unroll
      for (int by = 0; by < 4; ++by) {
        if (!((words[k] >> (8 * by)) & 1u)) continue;
        const uint32_t h = c * 16u + 4u * k + by;
        if (i < kListRun) {
          s_run[i] = h;
        } else {
          // past the run's capacity: straight to the frame list
          const uint32_t kk = atomicAdd(&m.st->f_count, 1u);
          if (kk < m.flist_cap) m.flist[kk] = h;
        }
        ++i;
      }
    }
  }
  __syncthreads();
  const uint32_t n = min(s_n, kListRun);
  if (threadIdx.x == 0) s_base = n ? atomicAdd(&m.st->f_count, n) : 0u;
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) {
    const uint32_t k = s_base + i;
    if (k < m.flist_cap) m.flist[k] = s_run[i];
  }
}

// Starts an allocation: empties the frame list and advances the allocation
// epoch.  Both live on the device, so a recorded launch sequence (a HIP graph
// of a frame) replays correctly.
__global__ void reset_frame_list_kernel(Batch b) {
  if (threadIdx.x == 0 && (int)blockIdx.x < b.n) {
    DevState* st = b.job[blockIdx.x].m.st;
    st->f_count = 0;
    advance_epoch(st);
  }
}

// ------------------------------------------------ compact free space
// (maps with free_blocks = 1; the free-space representation Sec. III-D
// leaves to future work, as coarse free-block flags.)  Before the
// integration every listed block is tested for being carved whole: its 8
// corner voxels, transformed as the integration transforms voxels, lie more
// than 1 mm in front of the camera and at least 1 mm before the clipping
// plane, the nearest pixels of their projections widened by one pixel span a
// rectangle inside the image of at most 64 depth cells (8x8 pixels), and
// every one of those cells holds a depth more than tau + 1 mm beyond the
// block's farthest corner (a cell: the smallest depth of its measured
// pixels; 0, failing the test, when a pixel is masked or none is measured).
// The voxels' depths and projections lie within the corners' range, far
// inside the margins, so with every pixel measured the per-voxel rule would
// carve every voxel of such a block; unmeasured pixels are carved over.
//
// A free block (no voxels, bucket slot kFreeSlot | count) carved whole only
// counts the frame, here, and is left out of the integration's work list.
// A free block not carved whole is evaluated by the integration voxel by
// voxel from its value (tau and its count, or unobserved while the count is
// 0): a band update gives it a pool slot, a frame that carves all of its
// voxels counts for it, any other frame leaves it as it is.  A block of
// voxels carved whole gives every voxel the free-space update without
// projecting it.  Work-list entries carry the outcome in bits 22-31 (bucket
// indices stay below 2^22).
constexpr uint32_t kEntryBucket = 0x003FFFFFu;
constexpr uint32_t kEntryWhole = 0x80000000u;  // carved whole
constexpr uint32_t kEntryFresh = 0x40000000u;  // a free block (alone: not carved whole, decided per voxel)
constexpr int kEntryCountShift = 22;           // the free block's count (bits 22-29)
constexpr float kCarveMargin = 1.0e-3f;        // metres
constexpr int kMaxTestCells = 64;
constexpr int kClassifyGroups = 512;           // workgroups of the whole-block test (all jobs together)

// One wavefront per 8x8 cell (lane = pixel), four cells per workgroup.  The
// first workgroup of a job also starts the frame's work list and its count
// of blocks carved whole (classify_kernel runs after it on the stream).
constexpr int kCellsPerGroup = 4;

template <int DF>
__global__ __launch_bounds__(256) void depth_cells_kernel(Batch b) {
  const int jb = batch_job(b, blockIdx.x);
  const Job& J = b.job[jb];
  const FrameDev& f = J.f;
  const int g = blockIdx.x - b.base[jb];
  if (g == 0 && threadIdx.x == 0) {
    J.m.st->w_count = 0;
    J.m.st->n_whole = 0;
  }
  const int c = g * kCellsPerGroup + (int)(threadIdx.x >> 6);
  if (c >= J.cells_w * J.cells_h) return;  // uniform per wavefront
  const int lane = threadIdx.x & 63;
  const int u = (c % J.cells_w) * kCell + (lane & 7), v = (c / J.cells_w) * kCell + (lane >> 3);
  const bool in = u < f.W && v < f.H;
  const int idx = in ? v * f.W + u : 0;
  const float D = in ? load_depth<DF>(f, idx) : 0.0f;
  const uint8_t* mask = J.mask;
  const bool masked = in && mask && mask[idx];
  float e = (D > 0.0f) ? D : INFINITY;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) e = fminf(e, __shfl_xor(e, o));
  const bool any_masked = __ballot(masked) != 0ull;
  if (lane == 0) J.m.cells[c] = (any_masked || e == INFINITY) ? 0.0f : e;
}

__device__ __forceinline__ bool carved_whole(const MapDev& m, const FrameDev& f, const Job& J, const float R[9],
                                             const float t[3], int bx, int by, int bz) {
  if (J.cells_w <= 0) return false;
  float zmin = INFINITY, zmax = -INFINITY, umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const float d0 = (float)(8 * bx + ((k & 1) ? 7 : 0)) * m.s - t[0];
    const float d1 = (float)(8 * by + ((k & 2) ? 7 : 0)) * m.s - t[1];
    const float d2 = (float)(8 * bz + ((k & 4) ? 7 : 0)) * m.s - t[2];
    const float x0 = (R[0] * d0 + R[3] * d1) + R[6] * d2;
    const float x1 = (R[1] * d0 + R[4] * d1) + R[7] * d2;
    const float x2 = (R[2] * d0 + R[5] * d1) + R[8] * d2;
    zmin = fminf(zmin, x2);
    zmax = fmaxf(zmax, x2);
    const float zz = fmaxf(x2, kCarveMargin);
    const float uf = f.fx * (x0 / zz) + f.cx, vf = f.fy * (x1 / zz) + f.cy;
    umin = fminf(umin, uf);
    umax = fmaxf(umax, uf);
    vmin = fminf(vmin, vf);
    vmax = fmaxf(vmax, vf);
  }
  if (!(zmin > kCarveMargin && zmax + kCarveMargin <= m.dmax)) return false;
  const float u0 = floorf(umin + 0.5f) - 1.0f, u1 = floorf(umax + 0.5f) + 1.0f;
  const float v0 = floorf(vmin + 0.5f) - 1.0f, v1 = floorf(vmax + 0.5f) + 1.0f;
  if (!(u0 >= 0.0f && v0 >= 0.0f && u1 <= (float)(f.W - 1) && v1 <= (float)(f.H - 1))) return false;
  const int c0 = (int)u0 / kCell, c1 = (int)u1 / kCell, r0 = (int)v0 / kCell, r1 = (int)v1 / kCell;
  if ((c1 - c0 + 1) * (r1 - r0 + 1) > kMaxTestCells) return false;
  float dmin = INFINITY;
  for (int r = r0; r <= r1; ++r)
    for (int c = c0; c <= c1; ++c) dmin = fminf(dmin, m.cells[r * J.cells_w + c]);
  return dmin > zmax + m.tau + kCarveMargin;
}

__global__ __launch_bounds__(256) void classify_kernel(Batch b) {
  const int jb = batch_job(b, blockIdx.x);
  const Job& J = b.job[jb];
  const MapDev& m = J.m;
  if (!m.free_blocks) return;
  const FrameDev& f = J.f;
  const uint32_t nF = min(m.st->f_count, m.flist_cap);
  const uint32_t g0 = blockIdx.x - b.base[jb], gn = b.base[jb + 1] - b.base[jb];
  float R[9], t[3];
  load_pose_f(J.pose, R, t);
  const uint32_t wmax = (uint32_t)m.max_weight;
  const int lane = threadIdx.x & 63;
  uint32_t n_whole = 0;
  // uniform trip count per workgroup, so every wavefront reaches the ballots
  const uint32_t step = gn * blockDim.x;
  for (uint32_t i0 = g0 * blockDim.x; i0 < nF; i0 += step) {
    const uint32_t i = i0 + threadIdx.x;
    bool work = false;
    uint32_t entry = 0;
    if (i < nF) {
      const uint32_t e = m.flist[i] & kEntryBucket;
      const Bucket bk = m.buckets[e];
      int bx, by, bz;
      unpack_key(bk.key, bx, by, bz);
      const bool whole = carved_whole(m, f, J, R, t, bx, by, bz);
      n_whole += whole;
      entry = e | (whole ? kEntryWhole : 0u);
      work = true;
      if (is_free_slot(bk.slot)) {
        const uint32_t c = bk.slot & 0xFFu;
        if (whole) {
          m.buckets[e].slot = kFreeSlot | min(c + 1u, wmax);
          work = false;  // a free block carved whole: counted, nothing left to do
        } else {
          entry |= kEntryFresh | (c << kEntryCountShift);  // free: decided voxel by voxel
        }
      }
    }
    // the entries left to the integration go to the work list, one atomic
    // per wavefront
    const unsigned long long bal = __ballot(work);
    if (bal != 0ull) {  // uniform
      const int leader = __ffsll((long long)bal) - 1;
      uint32_t base = 0;
      if (lane == leader) base = atomicAdd(&m.st->w_count, (uint32_t)__popcll(bal));
      base = __shfl(base, leader);
      const uint32_t pre = __builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
      if (work && base + pre < m.flist_cap) m.wlist[base + pre] = entry;
    }
  }
  __shared__ uint32_t s_whole;
  if (threadIdx.x == 0) s_whole = 0;
  __syncthreads();
  if (n_whole) atomicAdd(&s_whole, n_whole);
  __syncthreads();
  if (threadIdx.x == 0 && s_whole) atomicAdd(&m.st->n_whole, s_whole);
}

// Integration of one frame into the blocks of the frame list (Sec. III-A
// running average, Sec. III-D carving).  Workgroups stride over the list and
// take kIntegBlocks listed blocks per step; a thread owns voxels l and l + 256
// of each.  A workgroup's list entries and buckets (uniform) are read into
// LDS before its steps; a step issues the depth, the mask byte and the
// voxel record of every voxel together before any is used.  The record is
// read even for voxels the frame leaves untouched (about a fifth of a listed
// block), which costs those bytes but saves a dependent round trip; only
// voxels the frame updates are written.
constexpr int kIntegBlocks = 2;
constexpr int kIntegTab = 256;  // listed blocks a workgroup holds in LDS at a time

// COMPACT: some job of the batch keeps compact free space (its frame-list
// entries carry the whole-block test's outcome); without it those paths are
// compiled out.
template <int DF, int STORAGE, bool COMPACT>
__global__ __launch_bounds__(256) void integrate_kernel(Batch b) {
  constexpr int NV = 2 * kIntegBlocks;  // voxels per thread per step
  const int jb = batch_job(b, blockIdx.x);
  const Job& J = b.job[jb];
  // copies: the fields are read once, not at every use inside the branches
  const MapDev m = J.m;
  const FrameDev f = J.f;
  const uint8_t* mask = J.mask;
  const uint8_t* mask_src = mask ? mask : f.rgb;  // a readable plane when there is no mask
  const uint32_t g0 = blockIdx.x - b.base[jb], gn = b.base[jb + 1] - b.base[jb];
  // compact free-space maps work on the entries classify_kernel left (free
  // blocks carved whole are done), the others on the whole frame list
  const bool wl = COMPACT && m.free_blocks;
  const uint32_t* list = wl ? m.wlist : m.flist;
  const uint32_t nF = min(wl ? m.st->w_count : m.st->f_count, m.flist_cap);
  float R[9], t[3];
  load_pose_f(J.pose, R, t);
  uint32_t nb = 0, nf = 0;
  // correctly rounded reciprocals 1 / (W + 1) of the weights 0 .. 255
  __shared__ float s_rw[256];
  // compact free space: per pending free block of the step, its voxels'
  // decisions (bit 0 some band update, bit 1 some voxel not carved) and the
  // pool slot it takes
  __shared__ uint32_t s_pf[kIntegBlocks];
  __shared__ uint32_t s_pslot[kIntegBlocks];
  s_rw[threadIdx.x] = 1.0f / (float)(threadIdx.x + 1);
  if (threadIdx.x < kIntegBlocks) s_pf[threadIdx.x] = 0u;
  __syncthreads();
  // work-list entries of compact free-space maps carry the whole-block
  // test's outcome in their top bits (compact maps keep bucket indices below
  // 2^22); frame-list entries are plain bucket indices
  const uint32_t bucket_bits = wl ? kEntryBucket : 0xFFFFFFFFu;
  // The workgroup's listed blocks (entries g0, g0 + gn, ...) are read in
  // chunks of kIntegTab, list entries and then their buckets into LDS (two
  // round trips per chunk, the whole share of most workgroups), so a step
  // finds its blocks there and waits only on its voxel gathers.
  __shared__ unsigned long long s_tkey[kIntegTab];
  __shared__ uint32_t s_tslot[kIntegTab], s_tent[kIntegTab];
  const uint32_t nmine = g0 < nF ? (nF - g0 + gn - 1) / gn : 0u;  // entries of this workgroup
  for (uint32_t k0 = 0; k0 < nmine; k0 += kIntegTab) {
    const uint32_t nk = min(nmine - k0, (uint32_t)kIntegTab);
    __syncthreads();  // the previous chunk's steps are done with the table
    for (uint32_t q = threadIdx.x; q < nk; q += blockDim.x) {
      const uint32_t e = list[g0 + (k0 + q) * gn];
      const Bucket bq = m.buckets[e & bucket_bits];
      s_tkey[q] = bq.key;
      s_tslot[q] = bq.slot;
      s_tent[q] = e;
    }
    __syncthreads();
    for (uint32_t k = 0; k < nk; k += kIntegBlocks) {
      Bucket bu[kIntegBlocks];
      uint32_t st[kIntegBlocks];  // uniform: the whole-block test's outcome
      uint32_t eb[kIntegBlocks];  // uniform: bucket index
      bool live[kIntegBlocks], whole[kIntegBlocks], pend[kIntegBlocks];
#pragma unroll
      for (int i = 0; i < kIntegBlocks; ++i) {
        const bool in = k + i < nk;
        const uint32_t ki = in ? k + i : k;
        const uint32_t e = s_tent[ki];
        bu[i].key = s_tkey[ki];
        bu[i].slot = s_tslot[ki];
        st[i] = COMPACT ? (e & ~bucket_bits) : 0u;
        eb[i] = e & bucket_bits;
        whole[i] = (st[i] & kEntryWhole) != 0u;
        // a free block: evaluated voxel by voxel from its free value, it takes
        // a pool slot below if a voxel gets a band update
        pend[i] = (st[i] & (kEntryWhole | kEntryFresh)) == kEntryFresh;
        live[i] = in && (bu[i].slot < m.max_blocks || pend[i]);
      }
      int pix[NV];
      uint32_t vidx[NV];
      float X2[NV];
      bool vis[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int i = v >> 1;
        const int l = threadIdx.x + 256 * (v & 1);
        const bool ok = live[i];
        vidx[v] = (ok && !pend[i]) ? bu[i].slot * 512u + (uint32_t)l : 0u;
        if (whole[i]) {  // a block of voxels carved whole: no projection, no pixel
          pix[v] = 0;
          X2[v] = 0.0f;
          vis[v] = ok;
          continue;
        }
        int bx, by, bz;
        unpack_key(bu[i].key, bx, by, bz);
        // X = R^T (v s - t), summed as (R0j d0 + R1j d1) + R2j d2
        const float d0 = (float)(8 * bx + (l & 7)) * m.s - t[0];
        const float d1 = (float)(8 * by + ((l >> 3) & 7)) * m.s - t[1];
        const float d2 = (float)(8 * bz + (l >> 6)) * m.s - t[2];
        const float x0 = (R[0] * d0 + R[3] * d1) + R[6] * d2;
        const float x1 = (R[1] * d0 + R[4] * d1) + R[7] * d2;
        const float x2 = (R[2] * d0 + R[5] * d1) + R[8] * d2;
        bool in = ok && x2 > 0.0f;
        // x0 / x2 and x1 / x2 from one correctly rounded reciprocal (exact
        // quotients; x2 > 0 and the pixel test reject the rest)
        const float iz = 1.0f / x2;
        const float uf = f.fx * quotient_rn(x0, x2, iz) + f.cx;
        const float vf = f.fy * quotient_rn(x1, x2, iz) + f.cy;
        const float ur = floorf(uf + 0.5f), vr = floorf(vf + 0.5f);
        in = in && ur >= 0.0f && ur < (float)f.W && vr >= 0.0f && vr < (float)f.H;
        pix[v] = in ? (int)vr * f.W + (int)ur : 0;
        X2[v] = x2;
        vis[v] = in;
      }
      float D[NV], sdf[NV], W[NV];
      uint32_t mk[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        D[v] = 0.0f;
        mk[v] = 0u;
        if (!whole[v >> 1]) {
          D[v] = load_depth<DF>(f, pix[v]);
          mk[v] = mask_src[pix[v]];
        }
        if (!pend[v >> 1]) VoxelStore<STORAGE>::load(m, vidx[v], sdf[v], W[v]);
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) asm volatile("" : "+v"(D[v]), "+v"(mk[v]), "+v"(sdf[v]), "+v"(W[v]));
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (!pend[v >> 1]) continue;
        // a pending free block: every voxel starts from the free value (tau
        // and its count; unobserved while 0)
        const float c = (float)((st[v >> 1] >> kEntryCountShift) & 0xFFu);
        sdf[v] = c > 0.0f ? m.tau : 0.0f;
        W[v] = c;
      }
      // RN(1 / (W + 1)) of every voxel: from the table for the integral
      // weights the integration writes (0 .. 255), by division otherwise
      float rw[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int wi = (int)W[v];
        const bool tab = wi >= 0 && wi < 256 && (float)wi == W[v];
        rw[v] = s_rw[tab ? wi : 0];
        if (!tab) rw[v] = 1.0f / (W[v] + 1.0f);
      }
      // the per-voxel rule's decision and the new sdf of every voxel
      bool band[NV], upd[NV];
      float nsdf[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        band[v] = false;
        upd[v] = false;
        float dval = m.tau;
        if (whole[v >> 1]) {
          upd[v] = vis[v];  // carved whole: the free-space update
        } else if (vis[v] && D[v] > 0.0f && !(mask && mk[v])) {
          const float eta = D[v] - X2[v];
          if (eta >= -m.tau) {
            const bool bnd = eta <= m.tau;
            // the band of a measurement beyond depth_max is not integrated; the
            // free space in front of it is carved like any other (Sec. III-D)
            if (bnd ? (D[v] <= m.dmax) : (X2[v] <= m.dmax)) {
              upd[v] = true;
              band[v] = bnd;
              dval = bnd ? eta : m.tau;
            }
          }
        }
        nsdf[v] = quotient_rn(W[v] * sdf[v] + dval, W[v] + 1.0f, rw[v]);
      }
      // pending free blocks: a band update anywhere in the block gives it a pool
      // slot (all its voxels are then written); otherwise the frame counts for
      // the block if it carves every voxel of it, and leaves it as it is if not
      // (its value stands for space observed free in all of its voxels)
      bool fresh[kIntegBlocks];
#pragma unroll
      for (int i = 0; i < kIntegBlocks; ++i) fresh[i] = false;
      bool any_pend = false;
#pragma unroll
      for (int i = 0; i < kIntegBlocks; ++i) any_pend = any_pend || pend[i];
      if (COMPACT && any_pend) {  // uniform
#pragma unroll
        for (int v = 0; v < NV; ++v)
          if (pend[v >> 1] && live[v >> 1] && (band[v] || !upd[v])) atomicOr(&s_pf[v >> 1], band[v] ? 1u : 2u);
        __syncthreads();
        if (threadIdx.x < kIntegBlocks) {
          const int i = threadIdx.x;
          uint32_t slot = kInvalidSlot;
          if (pend[i] && live[i]) {
            const uint32_t fl = s_pf[i];
            const uint32_t c = (st[i] >> kEntryCountShift) & 0xFFu;
            if (fl & 1u) {
              slot = atomicAdd(&m.st->n_blocks, 1u);
              if (slot < m.max_blocks) {
                m.block_keys[slot] = bu[i].key;
              } else {
                slot = kInvalidSlot;
                atomicOr(&m.st->flags, (uint32_t)RF_FLAG_POOL_FULL);
              }
              m.buckets[eb[i]].slot = slot;
            } else if (!(fl & 2u)) {
              m.buckets[eb[i]].slot = kFreeSlot | min(c + 1u, (uint32_t)m.max_weight);
            }
          }
          s_pslot[i] = slot;
          s_pf[i] = 0u;
        }
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kIntegBlocks; ++i) {
          if (!pend[i]) continue;
          const uint32_t slot = s_pslot[i];
          fresh[i] = slot < m.max_blocks;
          if (fresh[i]) bu[i].slot = slot;
        }
#pragma unroll
        for (int v = 0; v < NV; ++v)
          if (fresh[v >> 1]) vidx[v] = bu[v >> 1].slot * 512u + (uint32_t)(threadIdx.x + 256 * (v & 1));
      }
      // stores: updated voxels; every voxel of a block that takes its pool slot now
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int i = v >> 1;
        if (pend[i] && !fresh[i]) {
          band[v] = false;  // stays a free block: nothing stored
          continue;
        }
        if (upd[v]) {
          VoxelStore<STORAGE>::store(m, vidx[v], nsdf[v], fminf(W[v] + 1.0f, m.max_weight));
          nb += band[v];
          nf += !band[v];
        } else if (fresh[i]) {
          VoxelStore<STORAGE>::store(m, vidx[v], sdf[v], W[v]);
        }
      }
      uint32_t cold[NV], cpx[NV][3];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        cold[v] = 0u;
        cpx[v][0] = cpx[v][1] = cpx[v][2] = 0u;
        if (!band[v]) continue;
        if (!fresh[v >> 1]) cold[v] = reinterpret_cast<const uint32_t*>(m.rgb)[vidx[v]];
        const uint8_t* px = f.rgb + 3 * pix[v];
        cpx[v][0] = px[0];
        cpx[v][1] = px[1];
        cpx[v][2] = px[2];
      }
#pragma unroll
      for (int v = 0; v < NV; ++v) asm volatile("" : "+v"(cold[v]), "+v"(cpx[v][0]), "+v"(cpx[v][1]), "+v"(cpx[v][2]));
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        if (!band[v]) continue;
        const float Wv = W[v], Wn = W[v] + 1.0f;
        float ch[3];
#pragma unroll
        for (int q = 0; q < 3; ++q)
          ch[q] = fminf(255.0f, fmaxf(0.0f, rintf(quotient_rn(
                                                Wv * (float)((cold[v] >> (8 * q)) & 0xFFu) + (float)cpx[v][q], Wn,
                                                rw[v]))));
        m.rgb[vidx[v]] = make_uchar4((unsigned char)ch[0], (unsigned char)ch[1], (unsigned char)ch[2], 0);
      }
    }
  }
  // per-workgroup update counts (band / free) for the roofline accounting:
  // each workgroup writes its own slot (one atomic per workgroup on a shared
  // counter would serialise ~1500 atomics per address), integ_fold_kernel sums
  __shared__ uint32_t s_cnt[2];
  if (threadIdx.x == 0) s_cnt[0] = s_cnt[1] = 0;
  __syncthreads();
  if (nb) atomicAdd(&s_cnt[0], nb);
  if (nf) atomicAdd(&s_cnt[1], nf);
  __syncthreads();
  if (threadIdx.x == 0) m.integ_counts[g0] = make_uint4(s_cnt[0], s_cnt[1], 0u, 0u);
}

// One workgroup per job: the integration's per-workgroup counts into the
// map's counters (last integration and cumulative).
__global__ __launch_bounds__(256) void integ_fold_kernel(Batch b) {
  const Job& J = b.job[blockIdx.x];
  const MapDev& m = J.m;
  const int ng = b.base[blockIdx.x + 1] - b.base[blockIdx.x];
  unsigned long long band = 0, free = 0;
  for (int i = threadIdx.x; i < ng; i += blockDim.x) {
    const uint4 c = m.integ_counts[i];
    band += c.x;
    free += c.y;
  }
  __shared__ unsigned long long s_b[256], s_f[256];
  s_b[threadIdx.x] = band;
  s_f[threadIdx.x] = free;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s_b[threadIdx.x] += s_b[threadIdx.x + w];
      s_f[threadIdx.x] += s_f[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    DevState* st = m.st;
    st->n_band = s_b[0];
    st->n_free = s_f[0];
    st->cum_band += s_b[0];
    st->cum_free += s_f[0];
    st->cum_blocks += min(st->f_count, m.flist_cap);
    st->cum_frames += 1;
    if (m.free_blocks) {
      // blocks carved whole, counted by classify_kernel
      st->cum_whole += st->n_whole;
      // free blocks changed their counts or took pool slots, so tracking
      // caches must not keep their old slot codes
      advance_epoch(st);
    }
  }
}

// ------------------------------------------------------------ host launchers
void launch_allocate(Batch& b, int depth_format, hipStream_t s) {
  reset_frame_list_kernel<<<b.n, 64, 0, s>>>(b);
  int total = 0;
  for (int j = 0; j < b.n; ++j) {
    Job& J = b.job[j];
    const int n = J.f.W * J.f.H;
    const int sc = (int)J.m.carve_stride;
    J.carve_w = (J.f.W + sc - 1) / sc;
    J.carve_h = (J.f.H + sc - 1) / sc;
    J.carve_groups = (J.carve_w * J.carve_h + 255) / 256;
    b.base[j] = total;
    total += J.carve_groups + (n + 255) / 256;
  }
  b.base[b.n] = total;
  if (depth_format == RF_DEPTH_U16) alloc_kernel<RF_DEPTH_U16><<<total, 256, 0, s>>>(b);
  else alloc_kernel<RF_DEPTH_F32><<<total, 256, 0, s>>>(b);
  const int per = kListGroups / b.n;
  for (int j = 0; j <= b.n; ++j) b.base[j] = j * per;
  list_frame_kernel<<<b.n * per, 256, 0, s>>>(b);
}

void launch_integrate(Batch& b, int depth_format, int storage, hipStream_t s) {
  // compact free-space maps: depth cells of the frame, then the whole-block
  // test of every listed block (a fixed share of workgroups per job; block
  // counts live on the device)
  int cells = 0;
  bool compact = false;
  for (int j = 0; j < b.n; ++j) {
    b.base[j] = cells;
    cells += (b.job[j].cells_w * b.job[j].cells_h + kCellsPerGroup - 1) / kCellsPerGroup;
    compact = compact || b.job[j].m.free_blocks;
  }
  b.base[b.n] = cells;
  if (compact) {
    if (cells > 0) {
      if (depth_format == RF_DEPTH_U16) depth_cells_kernel<RF_DEPTH_U16><<<cells, 256, 0, s>>>(b);
      else depth_cells_kernel<RF_DEPTH_F32><<<cells, 256, 0, s>>>(b);
    }
    const int per_c = kClassifyGroups / b.n;
    for (int j = 0; j <= b.n; ++j) b.base[j] = j * per_c;
    classify_kernel<<<b.n * per_c, 256, 0, s>>>(b);
  }
  // a fixed share of workgroups per job (block counts live on the device):
  // together one resident round (6 workgroups of 256 threads per CU)
  const int per = kIntegGroups / b.n;
  for (int j = 0; j <= b.n; ++j) b.base[j] = j * per;
  const int grid = b.n * per;
  auto run = [&](auto compact) {
    constexpr bool C = decltype(compact)::value;
    if (depth_format == RF_DEPTH_U16) {
      if (storage == RF_STORAGE_FP32) integrate_kernel<RF_DEPTH_U16, RF_STORAGE_FP32, C><<<grid, 256, 0, s>>>(b);
      else integrate_kernel<RF_DEPTH_U16, RF_STORAGE_FP16_U8, C><<<grid, 256, 0, s>>>(b);
    } else {
      if (storage == RF_STORAGE_FP32) integrate_kernel<RF_DEPTH_F32, RF_STORAGE_FP32, C><<<grid, 256, 0, s>>>(b);
      else integrate_kernel<RF_DEPTH_F32, RF_STORAGE_FP16_U8, C><<<grid, 256, 0, s>>>(b);
    }
  };
  if (compact) run(std::true_type{});
  else run(std::false_type{});
  integ_fold_kernel<<<b.n, 256, 0, s>>>(b);
}

}  // namespace rf
