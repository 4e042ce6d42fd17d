// Direct registration to the TSDF (Sec. III-B, Eqs. 1-4) for gfx950.
//
// One launch per Gauss-Newton/LM iteration.  Each thread evaluates pixels of
// the pyramid level (grid-stride), forms the depth residual S and the
// photometric residual Iv - I with their 6-DoF Jacobians in FP32, and
// accumulates the 29 normal-equation terms in FP64 (products of FP32 factors
// are exact in FP64).  Workgroups reduce with wavefront butterflies and LDS
// and write one FP64 partial each; the last workgroup to finish (agent-scope
// counter) sums the partials in a fixed order, solves the 6x6 system by
// Cholesky in FP64 and applies T <- exp(delta^) T to the device pose, so an
// iteration needs no host round trip and no second launch.
#include "rf_device.h"
#include "rf_internal.h"

namespace rf {

// ---------------------------------------------------------------- FP64 pose math
// Twist exponential: R = I + A K + B K^2, V = I + B K + C K^2, t = V rho.
__device__ void se3_exp_dev(const double xi[6], double E[12]) {
  const double p0 = xi[3], p1 = xi[4], p2 = xi[5];
  const double th2 = p0 * p0 + p1 * p1 + p2 * p2;
  double A, B, C;
  if (th2 < 1e-4) {
    const double t4 = th2 * th2, t6 = t4 * th2;
    A = 1.0 - th2 * (1.0 / 6.0) + t4 * (1.0 / 120.0) - t6 * (1.0 / 5040.0);
    B = 0.5 - th2 * (1.0 / 24.0) + t4 * (1.0 / 720.0) - t6 * (1.0 / 40320.0);
    C = (1.0 / 6.0) - th2 * (1.0 / 120.0) + t4 * (1.0 / 5040.0) - t6 * (1.0 / 362880.0);
  } else {
    const double th = sqrt(th2);
    const double sn = sin(th), hs = sin(0.5 * th);
    A = sn / th;
    B = 2.0 * hs * hs / th2;
    C = (th - sn) / (th2 * th);
  }
  // K = [phi]x ; K2 = phi phi^T - th2 I
  const double K[9] = {0, -p2, p1, p2, 0, -p0, -p1, p0, 0};
  const double ph[3] = {p0, p1, p2};
  double V[9];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      const double k2 = ph[i] * ph[j] - (i == j ? th2 : 0.0);
      const double id = (i == j) ? 1.0 : 0.0;
      E[4 * i + j] = id + A * K[3 * i + j] + B * k2;
      V[3 * i + j] = id + B * K[3 * i + j] + C * k2;
    }
  for (int i = 0; i < 3; ++i) E[4 * i + 3] = V[3 * i] * xi[0] + V[3 * i + 1] * xi[1] + V[3 * i + 2] * xi[2];
}

// Solves (H + lambda diag H) x = -g with H given by its 21 upper-triangle
// terms; false when a pivot is not above 1e-12 trace(H).
__device__ bool cholesky_solve6(const double ne[29], double lambda, double x[6]) {
  double L[6][6];
  double tr = 0.0;
  int k = 0;
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) {
      L[j][i] = ne[k++];  // lower triangle holds H
      if (i == j) tr += L[i][i];
    }
  for (int i = 0; i < 6; ++i) L[i][i] *= (1.0 + lambda);
  for (int c = 0; c < 6; ++c) {
    double piv = L[c][c];
    for (int q = 0; q < c; ++q) piv -= L[c][q] * L[c][q];
    if (!(piv > 1e-12 * tr)) return false;
    const double d = sqrt(piv);
    L[c][c] = d;
    const double inv = 1.0 / d;
    for (int r = c + 1; r < 6; ++r) {
      double a = L[r][c];
      for (int q = 0; q < c; ++q) a -= L[r][q] * L[c][q];
      L[r][c] = a * inv;
    }
  }
  double y[6];
  for (int r = 0; r < 6; ++r) {
    double a = -ne[21 + r];
    for (int q = 0; q < r; ++q) a -= L[r][q] * y[q];
    y[r] = a / L[r][r];
  }
  for (int r = 5; r >= 0; --r) {
    double a = y[r];
    for (int q = r + 1; q < 6; ++q) a -= L[q][r] * x[q];
    x[r] = a / L[r][r];
  }
  return true;
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

struct TrackArgs {
  int level;
  float w_c;
  int min_valid;
  double lm_lambda;
  int first_of_level;
  int mode;  // 0: solve and update the pose; 1: write the normal equations to out29
};

template <int DF, int STORAGE>
__global__ __launch_bounds__(kTrackBlock) void track_kernel(MapDev m, FrameDev f, const uint8_t* __restrict__ mask,
                                                            double* __restrict__ pose, TrackArgs a,
                                                            rf_track_stats* __restrict__ stats,
                                                            double* __restrict__ out29) {
  __shared__ int s_stop;
  __shared__ int s_last;
  __shared__ double s_wave[kTrackBlock / 64][32];
  __shared__ double s_grp[8][32];
  if (threadIdx.x == 0) s_stop = (a.mode == 0) ? (int)m.st->track_stop : 0;
  __syncthreads();
  if (s_stop) return;

  float R[9], t[3];
  load_pose_f(pose, R, t);
  const int lv = a.level;
  const int wl = (f.W + (1 << lv) - 1) >> lv;
  const int hl = (f.H + (1 << lv) - 1) >> lv;
  const int npx = wl * hl;
  const double wc = (double)a.w_c;

  double acc[kNE];
#pragma unroll
  for (int k = 0; k < kNE; ++k) acc[k] = 0.0;

  for (int i = blockIdx.x * kTrackBlock + threadIdx.x; i < npx; i += gridDim.x * kTrackBlock) {
    const int u = (i % wl) << lv, v = (i / wl) << lv;
    const int pix = v * f.W + u;
    const float D = load_depth<DF>(f, pix);
    if (!depth_ok(D, m.dmax)) continue;
    if (mask && mask[pix]) continue;
    const float x[3] = {(((float)u - f.cx) * f.ifx) * D, (((float)v - f.cy) * f.ify) * D, D};
    float y[3];
    xform(R, t, x, y);
    float S, gS[3], Iv, gI[3];
    if (!sample_map<STORAGE, true, true>(m, y, S, gS, Iv, gI)) continue;
    if (!(fabsf(S) < m.tau)) continue;
    const uint8_t* px = f.rgb + 3 * pix;
    const float rc = Iv - luminance((float)px[0], (float)px[1], (float)px[2]);
    const double Jd[6] = {gS[0], gS[1], gS[2], y[1] * gS[2] - y[2] * gS[1], y[2] * gS[0] - y[0] * gS[2],
                          y[0] * gS[1] - y[1] * gS[0]};
    const double Jc[6] = {gI[0], gI[1], gI[2], y[1] * gI[2] - y[2] * gI[1], y[2] * gI[0] - y[0] * gI[2],
                          y[0] * gI[1] - y[1] * gI[0]};
    const double rd = S, rcd = rc;
    int k = 0;
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      const double wJc = wc * Jc[r];
#pragma unroll
      for (int c = r; c < 6; ++c) {
        acc[k] = fma(Jd[r], Jd[c], acc[k]);
        acc[k] = fma(wJc, Jc[c], acc[k]);
        ++k;
      }
      acc[21 + r] = fma(Jd[r], rd, acc[21 + r]);
      acc[21 + r] = fma(wJc, rcd, acc[21 + r]);
    }
    acc[27] = fma(rd, rd, acc[27]);
    acc[27] = fma(wc * rcd, rcd, acc[27]);
    acc[28] += 1.0;
  }

  // workgroup reduction: wavefront butterflies, then the 4 wave sums in order
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < kNE; ++k) {
    const double v = wave_sum(acc[k]);
    if (lane == 0) s_wave[wave][k] = v;
  }
  __syncthreads();
  double* part = m.partials + (size_t)blockIdx.x * 32;
  if (threadIdx.x < kNE) {
    double v = 0.0;
#pragma unroll
    for (int w = 0; w < kTrackBlock / 64; ++w) v += s_wave[w][threadIdx.x];
    part[threadIdx.x] = v;
  }
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) s_last = (atomicAdd(&m.st->track_counter, 1u) == gridDim.x - 1);
  __syncthreads();
  if (!s_last) return;
  __threadfence();

  // last workgroup: fixed-order sum of the partials, 8 strided groups per term
  if (threadIdx.x < 8 * kNE) {
    const int c = threadIdx.x % kNE, g = threadIdx.x / kNE;
    double v = 0.0;
    for (int b = g; b < (int)gridDim.x; b += 8) v += m.partials[(size_t)b * 32 + c];
    s_grp[g][c] = v;
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  m.st->track_counter = 0;
  double ne[kNE];
  for (int c = 0; c < kNE; ++c) {
    double v = 0.0;
    for (int g = 0; g < 8; ++g) v += s_grp[g][c];
    ne[c] = v;
  }
  if (a.mode == 1) {
    for (int c = 0; c < kNE; ++c) out29[c] = ne[c];
    return;
  }
  if (stats) {
    stats->cost = ne[27];
    stats->count = ne[28];
    if (a.first_of_level && lv < 8) stats->level_count[lv] = ne[28];
  }
  uint32_t fl = 0;
  double delta[6];
  if (ne[28] < (double)a.min_valid) fl = RF_FLAG_TRACK_FEW_PIXELS;
  else if (!cholesky_solve6(ne, a.lm_lambda, delta)) fl = RF_FLAG_TRACK_SINGULAR;
  if (fl) {
    m.st->track_stop = 1;
    atomicOr(&m.st->flags, fl);
    if (stats) stats->flags |= fl;
    return;
  }
  double E[12], T[16];
  se3_exp_dev(delta, E);
  for (int i = 0; i < 16; ++i) T[i] = pose[i];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 4; ++j) {
      double v = E[4 * i] * T[j] + E[4 * i + 1] * T[4 + j] + E[4 * i + 2] * T[8 + j];
      if (j == 3) v += E[4 * i + 3];
      pose[4 * i + j] = v;
    }
  if (stats) stats->iters += 1;
}

__global__ void track_reset_kernel(MapDev m, rf_track_stats* stats) {
  if (threadIdx.x == 0) {
    m.st->track_stop = 0;
    m.st->track_counter = 0;
    if (stats) {
      stats->cost = 0.0;
      stats->count = 0.0;
      stats->iters = 0;
      stats->flags = 0;
      for (int l = 0; l < 8; ++l) stats->level_count[l] = 0.0;
    }
  }
}

static int track_grid(const FrameDev& f, int level) {
  const int wl = (f.W + (1 << level) - 1) >> level;
  const int hl = (f.H + (1 << level) - 1) >> level;
  const int g = (wl * hl + kTrackBlock - 1) / kTrackBlock;
  return g < 1 ? 1 : (g > kTrackMaxGroups ? kTrackMaxGroups : g);
}

template <int DF, int STORAGE>
static void track_launch(const MapDev& m, const FrameDev& f, const uint8_t* mask, double* pose, const TrackArgs& a,
                         rf_track_stats* stats, double* out29, hipStream_t s) {
  track_kernel<DF, STORAGE><<<track_grid(f, a.level), kTrackBlock, 0, s>>>(m, f, mask, pose, a, stats, out29);
}

static void track_dispatch(const MapDev& m, const FrameDev& f, int df, int st, const uint8_t* mask, double* pose,
                           const TrackArgs& a, rf_track_stats* stats, double* out29, hipStream_t s) {
  if (df == RF_DEPTH_U16) {
    if (st == RF_STORAGE_FP32) track_launch<RF_DEPTH_U16, RF_STORAGE_FP32>(m, f, mask, pose, a, stats, out29, s);
    else track_launch<RF_DEPTH_U16, RF_STORAGE_FP16_U8>(m, f, mask, pose, a, stats, out29, s);
  } else {
    if (st == RF_STORAGE_FP32) track_launch<RF_DEPTH_F32, RF_STORAGE_FP32>(m, f, mask, pose, a, stats, out29, s);
    else track_launch<RF_DEPTH_F32, RF_STORAGE_FP16_U8>(m, f, mask, pose, a, stats, out29, s);
  }
}

void launch_track(const MapDev& m, const FrameDev& f, int df, int st, const rf_track_params& tp,
                  const uint8_t* mask, double* pose, rf_track_stats* stats, hipStream_t s) {
  track_reset_kernel<<<1, 64, 0, s>>>(m, stats);
  for (int l = tp.levels - 1; l >= 0; --l)
    for (int it = 0; it < tp.iters_per_level; ++it) {
      TrackArgs a{l, tp.w_c, tp.min_valid, tp.lm_lambda, it == 0 ? 1 : 0, 0};
      track_dispatch(m, f, df, st, mask, pose, a, stats, nullptr, s);
    }
}

void launch_normal_equations(const MapDev& m, const FrameDev& f, int df, int st, const uint8_t* mask,
                             const double* pose, int level, float w_c, double* out29, hipStream_t s) {
  track_reset_kernel<<<1, 64, 0, s>>>(m, nullptr);
  TrackArgs a{level, w_c, 0, 0.0, 0, 1};
  track_dispatch(m, f, df, st, mask, const_cast<double*>(pose), a, nullptr, out29, s);
}

}  // namespace rf
