// Virtual depth by ray casting the model (Sec. III-E, second option for
// invalid measurements), for gfx950.
//
// One thread per pixel.  Along the pixel's ray the samples are taken at
// camera depths z_k = z_near + k step, step = tau / 2, at the back-projection
// of the pixel at z_k (Eq. 1) moved to the world by the pose; the virtual
// depth is the first crossing from a defined sample S_{k-1} > 0 to a defined
// sample S_k <= 0, z_{k-1} + step (S_{k-1} / (S_{k-1} - S_k)), or 0.  With
// only_invalid the pixels whose depth is not zero keep it (metres) and only
// the zeros are cast, getting the virtual depth or far_value.
//
// A thread keeps the pool slots of the 2x2x2 blocks above the block of a
// sample's lower corner, so the hash table is probed only when the ray
// enters a new block (about one sample in five); absent blocks are kept as
// -1.  The corner records of up to kRaySamples consecutive samples whose
// corners lie in that neighbourhood are loaded together (one round trip).
#include "rf_device.h"
#include "rf_internal.h"

namespace rf {

// Slot codes of blocks (bx + dx, by + dy, bz + dz), index dx + 2 dy + 4 dz;
// -1 if absent, <= -2 for a free block.  The 8 home buckets are read
// together (one round trip).
__device__ __forceinline__ void neighbourhood_slots(const MapDev& m, int bx, int by, int bz, int sl[8]) {
  unsigned long long bkey[8];
  uint32_t bslot[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const Bucket* p = m.buckets + (hash3(bx + (k & 1), by + ((k >> 1) & 1), bz + (k >> 2)) & m.bucket_mask);
    bkey[k] = p->key;
    bslot[k] = p->slot;
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int x = bx + (k & 1), y = by + ((k >> 1) & 1), z = bz + (k >> 2);
    Bucket b0;
    b0.key = bkey[k];
    b0.slot = bslot[k];
    sl[k] = resolve_slot(m, b0, pack_key(x, y, z), hash3(x, y, z) & m.bucket_mask);
  }
}

constexpr int kRaySamples = 2;  // samples whose corner records are loaded together (of 2, 4 and 8, 2 measured fastest)

template <int DF, int STORAGE>
__global__ __launch_bounds__(256) void raycast_kernel(MapDev m, FrameDev f, const double* pose, float z_near,
                                                      float z_far, float far_value, int only_invalid, float* out) {
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= f.W * f.H) return;
  const int u = idx % f.W, v = idx / f.W;
  const float D = only_invalid ? load_depth<DF>(f, idx) : 0.0f;  // the depth is read only to fill it
  if (only_invalid && D != 0.0f) {
    out[idx] = D;
    return;
  }
  float R[9], t[3];
  load_pose_f(pose, R, t);
  const float step = 0.5f * m.tau;
  const float ru = ((float)u - f.cx) * f.ifx, rv = ((float)v - f.cy) * f.ify;
  float hit = 0.0f, prev = 0.0f;
  bool have_prev = false;
  int base[3] = {INT_MIN, INT_MIN, INT_MIN};
  int sl[8];
  // Samples go in batches: the first sample of a batch fixes the 2x2x2 block
  // neighbourhood (probed if it changed), the batch runs on while the
  // following samples' corners stay inside it (at most kRaySamples), the
  // corner records of the whole batch are loaded together, and the batch's
  // samples are then tested in order, exactly as one at a time.
  int k = 0;
  while (true) {
    const float z0 = z_near + (float)k * step;
    if (!(z0 <= z_far)) break;
    int i0[kRaySamples][3];
    float fr[kRaySamples][3];
    bool ok[kRaySamples];
    int nb = 0;  // samples in this batch
#pragma unroll
    for (int q = 0; q < kRaySamples; ++q) {
      const float z = z_near + (float)(k + q) * step;
      const float x[3] = {ru * z, rv * z, z};
      float y[3];
      xform(R, t, x, y);
      ok[q] = (z <= z_far) && voxel_cell(m, y, i0[q], fr[q]);
      if (q == 0) {
        if (ok[0]) {
          const int b0[3] = {i0[0][0] >> 3, i0[0][1] >> 3, i0[0][2] >> 3};
          if (b0[0] != base[0] || b0[1] != base[1] || b0[2] != base[2]) {
            base[0] = b0[0];
            base[1] = b0[1];
            base[2] = b0[2];
            neighbourhood_slots(m, b0[0], b0[1], b0[2], sl);
          }
        }
        nb = 1;
      } else if (nb == q) {
        // corners of sample q inside the neighbourhood: (i0 >> 3) and ((i0 + 1) >> 3) - base in {0, 1}
        bool in = ok[q] && ok[0];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int lo = (i0[q][a] >> 3) - base[a], hi = ((i0[q][a] + 1) >> 3) - base[a];
          in = in && lo >= 0 && hi <= 1;
        }
        if (in) nb = q + 1;
      }
    }
    float cs[kRaySamples][8], cw[kRaySamples][8];
    bool got[kRaySamples];
#pragma unroll
    for (int q = 0; q < kRaySamples; ++q) {
      got[q] = q < nb && ok[q];
#pragma unroll
      for (int c = 0; c < 8; ++c) {
        const int dx = c & 1, dy = (c >> 1) & 1, dz = c >> 2;
        const int o = (((i0[q][0] + dx) >> 3) - base[0]) | ((((i0[q][1] + dy) >> 3) - base[1]) << 1) |
                      ((((i0[q][2] + dz) >> 3) - base[2]) << 2);
        const int s = got[q] ? sl[o & 7] : -1;
        got[q] = got[q] && s != -1;
        const uint32_t vi = (uint32_t)(s >= 0 ? s : 0) * 512u +
                            (uint32_t)(((i0[q][0] + dx) & 7) + 8 * ((i0[q][1] + dy) & 7) + 64 * ((i0[q][2] + dz) & 7));
        VoxelStore<STORAGE>::load(m, vi, cs[q][c], cw[q][c]);
        if (s <= -2) {  // free block (compact free space): (tau, count), unobserved while the count is 0
          const float fc = (float)(-2 - s);
          cs[q][c] = fc > 0.0f ? m.tau : 0.0f;
          cw[q][c] = fc;
        }
      }
    }
    bool done = false;
#pragma unroll
    for (int q = 0; q < kRaySamples; ++q) {
      if (done || q >= nb) continue;
      float S = 0.0f, gS[3], Iv, gI[3];
      uint32_t cc[8];
      const bool defined = got[q] && interpolate<false, false>(m, cs[q], cw[q], cc, fr[q], S, gS, Iv, gI);
      if (!defined) {
        have_prev = false;
        continue;
      }
      if (have_prev && prev > 0.0f && S <= 0.0f) {
        const float zp = z_near + (float)(k + q - 1) * step;
        hit = zp + step * (prev / (prev - S));
        done = true;
        continue;
      }
      prev = S;
      have_prev = true;
    }
    if (done) break;
    k += nb;
  }
  out[idx] = only_invalid ? (hit > 0.0f ? hit : far_value) : hit;
}

void launch_raycast(const MapDev& m, const FrameDev& f, int depth_format, int storage, const double* pose,
                    float z_near, float z_far, float far_value, int only_invalid, float* out, hipStream_t s) {
  const int n = f.W * f.H;
  const dim3 g((n + 255) / 256), blk(256);
  if (depth_format == RF_DEPTH_U16) {
    if (storage == RF_STORAGE_FP32)
      raycast_kernel<RF_DEPTH_U16, RF_STORAGE_FP32><<<g, blk, 0, s>>>(m, f, pose, z_near, z_far, far_value, only_invalid, out);
    else
      raycast_kernel<RF_DEPTH_U16, RF_STORAGE_FP16_U8><<<g, blk, 0, s>>>(m, f, pose, z_near, z_far, far_value, only_invalid,
                                                                        out);
  } else {
    if (storage == RF_STORAGE_FP32)
      raycast_kernel<RF_DEPTH_F32, RF_STORAGE_FP32><<<g, blk, 0, s>>>(m, f, pose, z_near, z_far, far_value, only_invalid, out);
    else
      raycast_kernel<RF_DEPTH_F32, RF_STORAGE_FP16_U8><<<g, blk, 0, s>>>(m, f, pose, z_near, z_far, far_value, only_invalid,
                                                                        out);
  }
}

}  // namespace rf
