// Block allocation (Sec. III-A, III-D) and TSDF integration with free-space
// carving (Sec. III-A, III-C, III-D) for gfx950.
//
// Allocation: one thread per pixel walks the block grid along its band (or
// carve) segment with a DDA; each visited block is inserted into the hash by
// CAS and, the first time it is touched in this frame (per-bucket frame
// stamp, exchanged atomically), appended to the frame's block list.  Carve
// rays run in workgroups of their own; cells are probed 8 at a time.
//
// Integration: one workgroup per listed block, 256 threads x 2 voxels; a
// voxel's record is read and written only when it is updated (occluded,
// masked and out-of-view voxels cost no HBM traffic).  Records are SoA per
// block, so a workgroup's loads and stores are contiguous 4-KiB (FP32) /
// 2-KiB (FP16) runs.
#include "rf_device.h"
#include "rf_internal.h"

namespace rf {

// Records a block of the frame: first touch this frame (stamp exchanged
// atomically) appends its bucket to the frame list.  stamp0 is the stamp
// value seen by the probe: equal to frame_id means already recorded.
__device__ __forceinline__ void touch_block(const MapDev& m, int h, uint32_t stamp0, uint32_t frame_id) {
  if (stamp0 == frame_id) return;
  if (atomicExch(&m.buckets[h].stamp, frame_id) != frame_id) {
    const uint32_t i = atomicAdd(&m.st->f_count, 1u);
    if (i < m.flist_cap) m.flist[i] = (uint32_t)h;
  }
}

// True for exactly one active lane per distinct key among the lanes with
// valid set (wavefront-level de-duplication: neighbouring rays visit the same
// blocks, and only one of them needs to probe, insert or stamp a block).
__device__ __forceinline__ bool wave_first_of_key(unsigned long long key, bool valid) {
  const int lane = threadIdx.x & 63;
  unsigned long long todo = __ballot(valid);
  bool leader = false;
  while (todo) {
    const int l = __ffsll((long long)todo) - 1;
    const unsigned int klo = __builtin_amdgcn_readlane((unsigned int)key, l);
    const unsigned int khi = __builtin_amdgcn_readlane((unsigned int)(key >> 32), l);
    const unsigned long long k = ((unsigned long long)khi << 32) | klo;
    todo &= ~__ballot(valid && key == k);
    leader |= (lane == l);
  }
  return leader;
}

// Block-grid DDA of segment q0 -> q1 (block units): cells c = floor(q0) ...
// e = floor(q1), exactly |e-c|_1 steps, each along the axis with the smallest
// next-boundary parameter among the axes not yet at e (ties: x, y, z).  Cells
// are produced in batches of 8 whose home buckets are loaded together, so a
// ray costs one hash round trip per 8 cells instead of one per cell.
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
  __device__ __forceinline__ void advance() {
    int best = -1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (c[a] == e[a]) continue;
      if (best < 0 || tmax[a] < tmax[best]) best = a;
    }
    c[best] += step[best];
    tmax[best] += tdel[best];
  }
};

template <int DF>
__global__ __launch_bounds__(256) void alloc_kernel(Batch b) {
  // Per job: workgroups [0, band_groups) take the band segments of the pixels
  // that are not on the carve grid; the rest take the carve segments of the
  // carve-grid pixels, so the long rays share wavefronts with rays of similar
  // length.
  const int jb = batch_job(b, blockIdx.x);
  const Job& J = b.job[jb];
  const MapDev& m = J.m;
  const FrameDev& f = J.f;
  const int g = blockIdx.x - b.base[jb];
  int u, v;
  const int s_c = (int)m.carve_stride;
  if (g < J.band_groups) {
    const int idx = g * blockDim.x + threadIdx.x;
    if (idx >= f.W * f.H) return;
    u = idx % f.W;
    v = idx / f.W;
    if (u % s_c == 0 && v % s_c == 0) return;
  } else {
    const int j = (g - J.band_groups) * blockDim.x + threadIdx.x;
    if (j >= J.carve_w * J.carve_h) return;
    u = (j % J.carve_w) * s_c;
    v = (j / J.carve_w) * s_c;
  }
  const uint8_t* mask = J.mask;
  const double* pose = J.pose;
  const uint32_t frame_id = J.frame_id;
  const int idx = v * f.W + u;
  const float D = load_depth<DF>(f, idx);
  if (!depth_ok(D, m.dmax)) return;
  if (mask && mask[idx]) return;
  float R[9], t[3];
  load_pose_f(pose, R, t);
  const bool carve = (u % s_c == 0) && (v % s_c == 0);
  const float zn = carve ? 0.0f : fmaxf(D - m.tau, 0.0f);
  const float zf = D + m.tau;
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
  constexpr int kBatch = 8;
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
    unsigned long long key[kBatch];
    uint32_t hb[kBatch];
    Bucket bk[kBatch];
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      key[q] = pack_key(cx[q], cy[q], cz[q]);
      ok[q] = wave_first_of_key(key[q], ok[q]);
      if (!ok[q]) continue;
      hb[q] = hash3(cx[q], cy[q], cz[q]) & m.bucket_mask;
      bk[q] = m.buckets[hb[q]];
    }
#pragma unroll
    for (int q = 0; q < kBatch; ++q) {
      if (!ok[q]) continue;
      if (bk[q].key == key[q]) {
        touch_block(m, (int)hb[q], bk[q].stamp, frame_id);
      } else {
        const int h = insert_block(m, cx[q], cy[q], cz[q]);
        if (h >= 0) touch_block(m, h, m.buckets[h].stamp, frame_id);
      }
    }
  }
}

__global__ void reset_frame_list_kernel(Batch b) {
  if (threadIdx.x == 0 && (int)blockIdx.x < b.n) {
    DevState* st = b.job[blockIdx.x].m.st;
    st->f_count = 0;
    st->n_band = 0;
    st->n_free = 0;
  }
}

// Integration of one frame into the blocks of the frame list: one
// workgroup per listed block at a time (grid-stride over the list), 256
// threads x 2 voxels; both voxels of a thread are independent, so their
// gathers overlap.  A voxel's record is read and written only when the frame
// updates it.
#ifndef RF_INTEG_SPEC
#define RF_INTEG_SPEC 0
#endif
// Returns 0 (untouched), 1 (band update) or 2 (free-space update).
template <int DF, int STORAGE>
__device__ __forceinline__ int integrate_voxel(const MapDev& m, const FrameDev& f, const uint8_t* mask,
                                               const float R[9], const float t[3], int bx, int by, int bz, int l,
                                               uint32_t vidx) {
#if RF_INTEG_SPEC
  float sdf, W;
  VoxelStore<STORAGE>::load(m, vidx, sdf, W);
#endif
  // X = R^T (v s - t), summed as (R0j d0 + R1j d1) + R2j d2
  const float d0 = (float)(8 * bx + (l & 7)) * m.s - t[0];
  const float d1 = (float)(8 * by + ((l >> 3) & 7)) * m.s - t[1];
  const float d2 = (float)(8 * bz + (l >> 6)) * m.s - t[2];
  const float X0 = (R[0] * d0 + R[3] * d1) + R[6] * d2;
  const float X1 = (R[1] * d0 + R[4] * d1) + R[7] * d2;
  const float X2 = (R[2] * d0 + R[5] * d1) + R[8] * d2;
  if (!(X2 > 0.0f)) return 0;
  const float uf = f.fx * (X0 / X2) + f.cx;
  const float vf = f.fy * (X1 / X2) + f.cy;
  const float ur = floorf(uf + 0.5f), vr = floorf(vf + 0.5f);
  if (!(ur >= 0.0f && ur < (float)f.W && vr >= 0.0f && vr < (float)f.H)) return 0;
  const int pix = (int)vr * f.W + (int)ur;
  const float D = load_depth<DF>(f, pix);
  if (!depth_ok(D, m.dmax)) return 0;
  if (mask && mask[pix]) return 0;
  const float eta = D - X2;
  if (eta < -m.tau) return 0;
  const bool band = (eta <= m.tau);
  if (!band && !(X2 <= m.dmax)) return 0;
  const float dval = band ? eta : m.tau;
#if !RF_INTEG_SPEC
  float sdf, W;
  VoxelStore<STORAGE>::load(m, vidx, sdf, W);
#endif
  const float Wn = W + 1.0f;
  VoxelStore<STORAGE>::store(m, vidx, (W * sdf + dval) / Wn, fminf(Wn, m.max_weight));
  if (band) {
    const uchar4 c = m.rgb[vidx];
    const uint8_t* px = f.rgb + 3 * pix;
    const float r = fminf(255.0f, fmaxf(0.0f, rintf((W * (float)c.x + (float)px[0]) / Wn)));
    const float g = fminf(255.0f, fmaxf(0.0f, rintf((W * (float)c.y + (float)px[1]) / Wn)));
    const float bl = fminf(255.0f, fmaxf(0.0f, rintf((W * (float)c.z + (float)px[2]) / Wn)));
    m.rgb[vidx] = make_uchar4((unsigned char)r, (unsigned char)g, (unsigned char)bl, 0);
    return 1;
  }
  return 2;
}

template <int DF, int STORAGE>
__global__ __launch_bounds__(256) void integrate_kernel(Batch b) {
  const int jb = batch_job(b, blockIdx.x);
  const Job& J = b.job[jb];
  const MapDev& m = J.m;
  const FrameDev& f = J.f;
  const uint8_t* mask = J.mask;
  const uint32_t g0 = blockIdx.x - b.base[jb], gn = b.base[jb + 1] - b.base[jb];
  const uint32_t nF = min(m.st->f_count, m.flist_cap);
  float R[9], t[3];
  load_pose_f(J.pose, R, t);
  uint32_t nb = 0, nf = 0;
  const int l0 = threadIdx.x, l1 = threadIdx.x + 256;
  for (uint32_t fi = g0; fi < nF; fi += gn) {
    const uint32_t h = m.flist[fi];
    const Bucket bu = m.buckets[h];
    if (bu.slot >= m.max_blocks) continue;
    int bx, by, bz;
    unpack_key(bu.key, bx, by, bz);
    const int r0 = integrate_voxel<DF, STORAGE>(m, f, mask, R, t, bx, by, bz, l0, bu.slot * 512u + (uint32_t)l0);
    const int r1 = integrate_voxel<DF, STORAGE>(m, f, mask, R, t, bx, by, bz, l1, bu.slot * 512u + (uint32_t)l1);
    nb += (r0 == 1) + (r1 == 1);
    nf += (r0 == 2) + (r1 == 2);
  }
  // per-workgroup update counts (band / free) for the roofline accounting
  __shared__ uint32_t s_cnt[2];
  if (threadIdx.x == 0) s_cnt[0] = s_cnt[1] = 0;
  __syncthreads();
  if (nb) atomicAdd(&s_cnt[0], nb);
  if (nf) atomicAdd(&s_cnt[1], nf);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (s_cnt[0]) {
      atomicAdd(&m.st->n_band, (unsigned long long)s_cnt[0]);
      atomicAdd(&m.st->cum_band, (unsigned long long)s_cnt[0]);
    }
    if (s_cnt[1]) {
      atomicAdd(&m.st->n_free, (unsigned long long)s_cnt[1]);
      atomicAdd(&m.st->cum_free, (unsigned long long)s_cnt[1]);
    }
    if (g0 == 0) {
      atomicAdd(&m.st->cum_blocks, (unsigned long long)nF);
      atomicAdd(&m.st->cum_frames, 1ull);
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
    J.band_groups = (n + 255) / 256;
    J.carve_w = (J.f.W + sc - 1) / sc;
    J.carve_h = (J.f.H + sc - 1) / sc;
    b.base[j] = total;
    total += J.band_groups + (J.carve_w * J.carve_h + 255) / 256;
  }
  b.base[b.n] = total;
  if (depth_format == RF_DEPTH_U16) alloc_kernel<RF_DEPTH_U16><<<total, 256, 0, s>>>(b);
  else alloc_kernel<RF_DEPTH_F32><<<total, 256, 0, s>>>(b);
}

void launch_integrate(Batch& b, int depth_format, int storage, hipStream_t s) {
  // a fixed share of workgroups per job (block counts live on the device)
  const int per = b.n == 1 ? 2048 : (b.n <= 4 ? 1024 : 512);
  for (int j = 0; j <= b.n; ++j) b.base[j] = j * per;
  const int grid = b.n * per;
  if (depth_format == RF_DEPTH_U16) {
    if (storage == RF_STORAGE_FP32) integrate_kernel<RF_DEPTH_U16, RF_STORAGE_FP32><<<grid, 256, 0, s>>>(b);
    else integrate_kernel<RF_DEPTH_U16, RF_STORAGE_FP16_U8><<<grid, 256, 0, s>>>(b);
  } else {
    if (storage == RF_STORAGE_FP32) integrate_kernel<RF_DEPTH_F32, RF_STORAGE_FP32><<<grid, 256, 0, s>>>(b);
    else integrate_kernel<RF_DEPTH_F32, RF_STORAGE_FP16_U8><<<grid, 256, 0, s>>>(b);
  }
}

}  // namespace rf
