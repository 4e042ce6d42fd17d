// Block allocation (Sec. III-A, III-D) and TSDF integration with free-space
// carving (Sec. III-A, III-C, III-D) for gfx950.
//
// Allocation: one thread per pixel walks the block grid along its band (or
// carve) segment with a DDA; each visited block is inserted into the hash by
// CAS and, the first time it is touched in this frame (per-bucket frame
// stamp, exchanged atomically), appended to the frame's block list.
//
// Integration: one workgroup per listed block, 256 threads x 2 voxels; the
// keep/skip decision needs only the frame, so a voxel's record is read and
// written only when it is updated (occluded, masked and out-of-view voxels
// cost no HBM traffic).  Records are SoA per block, so a workgroup's loads
// and stores are contiguous 2-KiB (FP32) / 1-KiB (FP16) runs.
#include "rf_device.h"
#include "rf_internal.h"

namespace rf {

// Visit the block cells of segment q0 -> q1 (block units): exactly |e-c|_1
// steps, each along the axis with the smallest next-boundary parameter among
// the axes not yet at the end cell (ties: x, y, z).
template <typename Visit>
__device__ __forceinline__ void dda_blocks(const float q0[3], const float q1[3], Visit&& visit) {
  int c[3], e[3], step[3];
  float tmax[3], tdel[3];
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
  visit(c);
  for (int k = 0; k < n; ++k) {
    int best = -1;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (c[a] == e[a]) continue;
      if (best < 0 || tmax[a] < tmax[best]) best = a;
    }
    c[best] += step[best];
    tmax[best] += tdel[best];
    visit(c);
  }
}

template <int DF>
__global__ __launch_bounds__(256) void alloc_kernel(MapDev m, FrameDev f, const double* __restrict__ pose,
                                                    const uint8_t* __restrict__ mask, uint32_t frame_id) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= f.W * f.H) return;
  const int u = idx % f.W, v = idx / f.W;
  const float D = load_depth<DF>(f, idx);
  if (!depth_ok(D, m.dmax)) return;
  if (mask && mask[idx]) return;
  float R[9], t[3];
  load_pose_f(pose, R, t);
  const bool carve = (u % (int)m.carve_stride == 0) && (v % (int)m.carve_stride == 0);
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
  dda_blocks(q0, q1, [&](const int* c) {
    const int h = insert_block(m, c[0], c[1], c[2]);
    if (h < 0) return;
    uint32_t* stamp = &m.buckets[h].stamp;
    if (*stamp != frame_id) {
      if (atomicExch(stamp, frame_id) != frame_id) {
        const uint32_t i = atomicAdd(&m.st->f_count, 1u);
        if (i < m.flist_cap) m.flist[i] = (uint32_t)h;
      }
    }
  });
}

__global__ void reset_frame_list_kernel(MapDev m) {
  if (threadIdx.x == 0) {
    m.st->f_count = 0;
    m.st->n_band = 0;
    m.st->n_free = 0;
  }
}

// Integration of one frame into the blocks of the frame list.
template <int DF, int STORAGE>
__global__ __launch_bounds__(256) void integrate_kernel(MapDev m, FrameDev f, const double* __restrict__ pose,
                                                        const uint8_t* __restrict__ mask) {
  const uint32_t nF = min(m.st->f_count, m.flist_cap);
  float R[9], t[3];
  load_pose_f(pose, R, t);
  uint32_t nb = 0, nf = 0;
  for (uint32_t fi = blockIdx.x; fi < nF; fi += gridDim.x) {
    const uint32_t h = m.flist[fi];
    const uint32_t slot = m.buckets[h].slot;
    if (slot >= m.max_blocks) continue;
    int bx, by, bz;
    unpack_key(m.buckets[h].key, bx, by, bz);
    for (int l = threadIdx.x; l < 512; l += blockDim.x) {
      const int vi[3] = {8 * bx + (l & 7), 8 * by + ((l >> 3) & 7), 8 * bz + (l >> 6)};
      float d[3], X[3];
#pragma unroll
      for (int a = 0; a < 3; ++a) d[a] = (float)vi[a] * m.s - t[a];
#pragma unroll
      for (int j = 0; j < 3; ++j) X[j] = (R[j] * d[0] + R[3 + j] * d[1]) + R[6 + j] * d[2];
      if (!(X[2] > 0.0f)) continue;
      const float uf = f.fx * (X[0] / X[2]) + f.cx;
      const float vf = f.fy * (X[1] / X[2]) + f.cy;
      const float ur = floorf(uf + 0.5f), vr = floorf(vf + 0.5f);
      if (!(ur >= 0.0f && ur < (float)f.W && vr >= 0.0f && vr < (float)f.H)) continue;
      const int pix = (int)vr * f.W + (int)ur;
      const float D = load_depth<DF>(f, pix);
      if (!depth_ok(D, m.dmax)) continue;
      if (mask && mask[pix]) continue;
      const float eta = D - X[2];
      if (eta < -m.tau) continue;
      const bool band = (eta <= m.tau);
      if (!band && !(X[2] <= m.dmax)) continue;
      const float dval = band ? eta : m.tau;
      const uint32_t vidx = slot * 512u + (uint32_t)l;
      float sdf, W;
      VoxelStore<STORAGE>::load(m, vidx, sdf, W);
      const float Wn = W + 1.0f;
      VoxelStore<STORAGE>::store(m, vidx, (W * sdf + dval) / Wn, fminf(Wn, m.max_weight));
      if (band) {
        const uchar4 c = m.rgb[vidx];
        const uint8_t* px = f.rgb + 3 * pix;
        const float r = fminf(255.0f, fmaxf(0.0f, rintf((W * (float)c.x + (float)px[0]) / Wn)));
        const float g = fminf(255.0f, fmaxf(0.0f, rintf((W * (float)c.y + (float)px[1]) / Wn)));
        const float b = fminf(255.0f, fmaxf(0.0f, rintf((W * (float)c.z + (float)px[2]) / Wn)));
        m.rgb[vidx] = make_uchar4((unsigned char)r, (unsigned char)g, (unsigned char)b, 0);
        ++nb;
      } else {
        ++nf;
      }
    }
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
    if (blockIdx.x == 0) {
      atomicAdd(&m.st->cum_blocks, (unsigned long long)nF);
      atomicAdd(&m.st->cum_frames, 1ull);
    }
  }
}

// ------------------------------------------------------------ host launchers
void launch_allocate(const MapDev& m, const FrameDev& f, int depth_format, const double* pose,
                     const uint8_t* mask, uint32_t frame_id, hipStream_t s) {
  reset_frame_list_kernel<<<1, 64, 0, s>>>(m);
  const int n = f.W * f.H;
  const int grid = (n + 255) / 256;
  if (depth_format == RF_DEPTH_U16)
    alloc_kernel<RF_DEPTH_U16><<<grid, 256, 0, s>>>(m, f, pose, mask, frame_id);
  else
    alloc_kernel<RF_DEPTH_F32><<<grid, 256, 0, s>>>(m, f, pose, mask, frame_id);
}

int integrate_grid() { return 2048; }

void launch_integrate(const MapDev& m, const FrameDev& f, int depth_format, int storage, const double* pose,
                      const uint8_t* mask, hipStream_t s) {
  const int grid = integrate_grid();
  if (depth_format == RF_DEPTH_U16) {
    if (storage == RF_STORAGE_FP32)
      integrate_kernel<RF_DEPTH_U16, RF_STORAGE_FP32><<<grid, 256, 0, s>>>(m, f, pose, mask);
    else
      integrate_kernel<RF_DEPTH_U16, RF_STORAGE_FP16_U8><<<grid, 256, 0, s>>>(m, f, pose, mask);
  } else {
    if (storage == RF_STORAGE_FP32)
      integrate_kernel<RF_DEPTH_F32, RF_STORAGE_FP32><<<grid, 256, 0, s>>>(m, f, pose, mask);
    else
      integrate_kernel<RF_DEPTH_F32, RF_STORAGE_FP16_U8><<<grid, 256, 0, s>>>(m, f, pose, mask);
  }
}

}  // namespace rf
