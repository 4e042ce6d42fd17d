// ReFusion per-frame hot path: plain CPU ORACLE.
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
// load this file; only the tests, the smoke check and the benchmark's
// CPU-baseline leg use it.  It shares no code, header, table or helper with
// the GPU library: everything here is written from the paper (ReFusion,
// Palazzolo et al., IROS 2019) and the readings listed below.
//
// Style: slow and obvious.  Blocks live in a std::unordered_map keyed by the
// integer block coordinate; every loop is scalar; there is no blocking,
// fusion or reordering.  Values are computed in the template type Real
// (double for the FP64 reference; float for the FP32 mirror).  Where a
// floating-point value decides an integer (which pixel a voxel projects to,
// which block cells a ray visits, whether a residual exceeds the threshold)
// the decision is always taken in FP32 with the operation order spelled out in
// the comments, because that is the precision the GPU kernels decide in.
//
// Readings of points the paper leaves open (each repeated where it is used):
//  * voxel v in Z^3 has its centre at v*s; block = floor(v/8); local index
//    lx + 8 ly + 64 lz.
//  * pose T is camera->world, row-major 4x4; minimal update xi = (rho, phi),
//    translation first, applied on the left: T <- exp(xi^) T.
//  * trilinear sample is defined only where all 8 corner voxels exist with
//    weight > 0; gradient = exact derivative of the interpolant.
//  * tracking uses a sample only if |S| < tau (the dynamic mask uses every
//    defined sample).
//  * least squares solved by Gauss-Newton (LM with lambda = 0 unless given),
//    6x6 Cholesky in FP64; pyramid level l takes every 2^l-th pixel.
//  * allocation: band segment z in [max(D-tau,0), D+tau] for every valid
//    unmasked pixel, carve segment z in [0, D+tau] on a carve_stride pixel grid;
//    a block-grid DDA visits the cells of each segment.  A measurement beyond
//    depth_max (the clipping plane) is not valid for registration, the mask or
//    the band, but its carve segment z in [0, depth_max] is walked.
//  * integration: nearest-pixel projection, eta = D - z (optical axis), band
//    |eta| <= tau and D <= depth_max -> d = eta (and colour), eta > tau and
//    z <= depth_max -> d = tau (free space, also in front of measurements
//    beyond depth_max), otherwise untouched; observation weight 1, weight cap
//    max_weight; colour rounded half-to-even.
#include <algorithm>
#include <array>
#include <cmath>
#include <type_traits>
#include <cstdint>
#include <cstring>
#include <deque>
#include <limits>
#include <unordered_map>
#include <unordered_set>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <vector>

namespace {

// --------------------------------------------------------------------------
// keys and containers
// --------------------------------------------------------------------------
struct Key {
  int32_t x, y, z;
  bool operator==(const Key& o) const { return x == o.x && y == o.y && z == o.z; }
  bool operator<(const Key& o) const {
    if (x != o.x) return x < o.x;
    if (y != o.y) return y < o.y;
    return z < o.z;
  }
};
struct KeyHash {
  size_t operator()(const Key& k) const {
    uint64_t h = (uint64_t)(uint32_t)k.x * 0x9E3779B97F4A7C15ull;
    h ^= (uint64_t)(uint32_t)k.y * 0xC2B2AE3D27D4EB4Full + (h << 6) + (h >> 2);
    h ^= (uint64_t)(uint32_t)k.z * 0x165667B19E3779F9ull + (h << 6) + (h >> 2);
    return (size_t)h;
  }
};

inline int32_t floor_div8(int32_t v) { return (v >= 0) ? v / 8 : -((-v + 7) / 8); }

// --------------------------------------------------------------------------
// FP16 rounding (IEEE binary16, round to nearest, ties to even), written from
// the format's definition: 11 significant bits, minimum normal exponent -14.
// Used only by the FP16-storage mirror.
// --------------------------------------------------------------------------
float round_to_half(float x) {
  if (x == 0.0f || !std::isfinite(x)) return x;
  int ex;
  double m = std::frexp((double)x, &ex);  // |x| = |m| 2^ex, |m| in [0.5,1)
  (void)m;
  int e = ex - 1;                          // |x| in [2^e, 2^(e+1))
  if (e < -14) e = -14;                    // subnormal spacing below 2^-14
  double ulp = std::ldexp(1.0, e - 10);
  double q = std::nearbyint((double)x / ulp);  // exact quotient, RNE
  double r = q * ulp;
  if (std::fabs(r) >= 65520.0) return std::copysign(INFINITY, x);
  return (float)r;
}

// --------------------------------------------------------------------------
// Pose helpers (FP64).  Section III-B: T in SE(3), xi in se(3), exp map.
// --------------------------------------------------------------------------
void mat_identity(double* T) {
  for (int i = 0; i < 16; ++i) T[i] = (i % 5 == 0) ? 1.0 : 0.0;
}

// exp of the twist xi = (rho, phi): R = I + A K + B K^2, V = I + B K + C K^2,
// t = V rho, with K = [phi]x, theta = |phi|, A = sin/theta, B = (1-cos)/theta^2,
// C = (theta - sin)/theta^3 (series for small theta).
void se3_exp(const double* xi, double* T) {
  const double* rho = xi;
  const double* phi = xi + 3;
  double th2 = phi[0]*phi[0] + phi[1]*phi[1] + phi[2]*phi[2];
  double th = std::sqrt(th2);
  double A, B, C;
  if (th < 1e-2) {
    double t4 = th2*th2, t6 = t4*th2;
    A = 1.0 - th2/6.0 + t4/120.0 - t6/5040.0;
    B = 0.5 - th2/24.0 + t4/720.0 - t6/40320.0;
    C = 1.0/6.0 - th2/120.0 + t4/5040.0 - t6/362880.0;
  } else {
    double s = std::sin(th), h = std::sin(0.5*th);
    A = s/th;
    B = 2.0*h*h/th2;
    C = (th - s)/(th2*th);
  }
  double K[3][3] = {{0, -phi[2], phi[1]}, {phi[2], 0, -phi[0]}, {-phi[1], phi[0], 0}};
  double K2[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double acc = 0;
      for (int k = 0; k < 3; ++k) acc += K[i][k]*K[k][j];
      K2[i][j] = acc;
    }
  mat_identity(T);
  double V[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double I = (i == j) ? 1.0 : 0.0;
      T[4*i+j] = I + A*K[i][j] + B*K2[i][j];
      V[i][j] = I + B*K[i][j] + C*K2[i][j];
    }
  for (int i = 0; i < 3; ++i) T[4*i+3] = V[i][0]*rho[0] + V[i][1]*rho[1] + V[i][2]*rho[2];
}

// T <- exp(xi^) T   (left update)
void pose_left_update(const double* xi, double* T) {
  double E[16], N[16];
  se3_exp(xi, E);
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      double acc = 0;
      for (int k = 0; k < 4; ++k) acc += E[4*i+k]*T[4*k+j];
      N[4*i+j] = acc;
    }
  std::memcpy(T, N, sizeof(N));
}

// --------------------------------------------------------------------------
// Frame access.  Section III-B: D(p) depth, I(p) intensity,
// I = 0.2126 R + 0.7152 G + 0.0722 B (RGB scaled to [0,1]).
// --------------------------------------------------------------------------
struct Frame {
  int W, H;
  float fx, fy, cx, cy;
  const void* depth;
  int depth_u16;
  float depth_scale;
  const uint8_t* rgb;
};

// Depth in metres as FP32: u16 input is raw * scale in FP32; f32 input as is.
inline float depth_at(const Frame& f, int u, int v) {
  size_t i = (size_t)v*f.W + u;
  if (f.depth_u16) return (float)((const uint16_t*)f.depth)[i] * f.depth_scale;
  return ((const float*)f.depth)[i];
}
inline bool depth_valid(float D, float dmax) { return D > 0.0f && D <= dmax; }

template <class Real>
inline Real luminance(const uint8_t* c) {
  // ((0.2126 R + 0.7152 G) + 0.0722 B) / 255 (Sec. III-B: intensity of the
  // RGB colour, scaled to [0, 1]); a correctly rounded division in Real
  const Real x = (Real)0.2126f*(Real)c[0] + (Real)0.7152f*(Real)c[1] + (Real)0.0722f*(Real)c[2];
  return x / (Real)255.0f;
}

// --------------------------------------------------------------------------
// The map.  Section III-A: voxels hold SDF (positive in front of the surface),
// weight and colour; blocks of 8^3 voxels are allocated on demand and found
// through a spatial hash (here: std::unordered_map).
// --------------------------------------------------------------------------
struct Params {
  float voxel_size, truncation, depth_max;
  int max_weight, carve_stride;
  int storage;      // 0: Real; 1: mirror of FP16 sdf/tau + u8 weight storage
  int free_blocks;  // 1: compact free space (blocks carved whole, free blocks without voxels)
};

struct MapBase {
  virtual ~MapBase() {}
  Params P;
  std::vector<Key> last_F;  // blocks visited by the last allocation
  std::unordered_set<Key, KeyHash> F_set;
  virtual int64_t num_blocks() const = 0;
  virtual int64_t num_voxel_blocks() const = 0;
  virtual bool has_block(const Key& k) const = 0;
  virtual void add_block(const Key& k) = 0;
};

template <class Real>
struct Voxel {
  Real sdf = 0;
  Real w = 0;
  uint8_t rgb[3] = {0, 0, 0};
};

// Compact free space (P.free_blocks = 1; the octree or free-space
// representation that Sec. III-D leaves to future work, read here as coarse
// free-block flags): a new block is a free block, kept as one voxel value
// (sdf tau, weight = the number of frames that carved all of its voxels,
// capped; unobserved while that is 0) that every one of its 512 voxels reads
// as.  It becomes an ordinary block of voxels, all starting from that value,
// the first time one of its voxels gets a band update; a frame that carves
// only some of its voxels leaves it as it is.
template <class Real>
struct Map : MapBase {
  std::unordered_map<Key, std::vector<Voxel<Real>>, KeyHash> blocks;
  std::unordered_map<Key, Voxel<Real>, KeyHash> free_blk;  // free blocks (P.free_blocks)
  int64_t num_blocks() const override { return (int64_t)(blocks.size() + free_blk.size()); }
  int64_t num_voxel_blocks() const override { return (int64_t)blocks.size(); }
  bool has_block(const Key& k) const override { return blocks.count(k) != 0 || free_blk.count(k) != 0; }
  void add_block(const Key& k) override {
    if (has_block(k)) return;
    if (P.free_blocks) free_blk.emplace(k, Voxel<Real>());
    else blocks.emplace(k, std::vector<Voxel<Real>>(512));
  }
  const Voxel<Real>* voxel(int32_t vx, int32_t vy, int32_t vz) const {
    Key k{floor_div8(vx), floor_div8(vy), floor_div8(vz)};
    auto it = blocks.find(k);
    if (it == blocks.end()) {
      auto jt = free_blk.find(k);
      return jt == free_blk.end() ? nullptr : &jt->second;
    }
    int lx = vx - 8*k.x, ly = vy - 8*k.y, lz = vz - 8*k.z;
    return &it->second[lx + 8*ly + 64*lz];
  }
  // stored value as it reads back (FP16 mirror: decode of the rounded code)
  Real store_sdf(Real x) const {
    if (P.storage == 1) {
      float inv_tau = 1.0f / P.truncation;
      float code = round_to_half((float)x * inv_tau);
      return (Real)(code * P.truncation);
    }
    return x;
  }
};

// --------------------------------------------------------------------------
// Trilinear interpolation of SDF and intensity (Section III-B), with the
// exact gradient of the interpolant.  g = y / s (as y * (1/s)), i0 = floor(g),
// f = g - i0; lerp(a,b,t) = a + t (b - a) along x, then y, then z.
// --------------------------------------------------------------------------
template <class Real>
struct Sample {
  bool ok = false;
  Real S = 0, gS[3] = {0, 0, 0};
  Real Iv = 0, gI[3] = {0, 0, 0};
};

template <class Real>
inline Real lerp(Real a, Real b, Real t) { return a + t*(b - a); }

// Interpolates the 8 corner values c[dz][dy][dx]; returns value and d/dg.
template <class Real>
void trilinear(const Real c[2][2][2], const Real f[3], Real& val, Real grad_g[3]) {
  Real cx[2][2], dx[2][2];
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy) {
      cx[dz][dy] = lerp(c[dz][dy][0], c[dz][dy][1], f[0]);
      dx[dz][dy] = c[dz][dy][1] - c[dz][dy][0];
    }
  Real cy[2], dxy[2], dy[2];
  for (int dz = 0; dz < 2; ++dz) {
    cy[dz] = lerp(cx[dz][0], cx[dz][1], f[1]);
    dxy[dz] = lerp(dx[dz][0], dx[dz][1], f[1]);
    dy[dz] = cx[dz][1] - cx[dz][0];
  }
  val = lerp(cy[0], cy[1], f[2]);
  grad_g[0] = lerp(dxy[0], dxy[1], f[2]);
  grad_g[1] = lerp(dy[0], dy[1], f[2]);
  grad_g[2] = cy[1] - cy[0];
}

template <class Real>
Sample<Real> sample_at(const Map<Real>& m, const Real y[3]) {
  Sample<Real> out;
  const Real is = (Real)1 / (Real)m.P.voxel_size;
  Real g[3], f[3];
  int32_t i0[3];
  for (int a = 0; a < 3; ++a) {
    g[a] = y[a]*is;
    Real fl = std::floor(g[a]);
    if (!(fl > -1e9 && fl < 1e9)) return out;
    i0[a] = (int32_t)fl;
    f[a] = g[a] - fl;
  }
  Real cs[2][2][2], ci[2][2][2];
  for (int dz = 0; dz < 2; ++dz)
    for (int dy = 0; dy < 2; ++dy)
      for (int dx = 0; dx < 2; ++dx) {
        const Voxel<Real>* v = m.voxel(i0[0] + dx, i0[1] + dy, i0[2] + dz);
        if (!v || !(v->w > 0)) return out;
        cs[dz][dy][dx] = v->sdf;
        ci[dz][dy][dx] = luminance<Real>(v->rgb);
      }
  Real gs[3], gi[3];
  trilinear(cs, f, out.S, gs);
  trilinear(ci, f, out.Iv, gi);
  for (int a = 0; a < 3; ++a) {
    out.gS[a] = gs[a]*is;
    out.gI[a] = gi[a]*is;
  }
  out.ok = true;
  return out;
}

// y = R x + t, summed as ((R0 x0 + R1 x1) + R2 x2) + t
template <class Real>
inline void transform(const Real R[9], const Real t[3], const Real x[3], Real y[3]) {
  for (int i = 0; i < 3; ++i) y[i] = ((R[3*i]*x[0] + R[3*i+1]*x[1]) + R[3*i+2]*x[2]) + t[i];
}

template <class Real>
void pose_split(const double* T, Real R[9], Real t[3]) {
  for (int i = 0; i < 3; ++i) {
    for (int j = 0; j < 3; ++j) R[3*i+j] = (Real)T[4*i+j];
    t[i] = (Real)T[4*i+3];
  }
}

// Eq. (1): x = ((u-cx)/fx D, (v-cy)/fy D, D), evaluated as ((u-cx) * (1/fx)) * D.
template <class Real>
void backproject(const Frame& f, int u, int v, Real D, Real x[3]) {
  const Real ifx = (Real)1 / (Real)f.fx, ify = (Real)1 / (Real)f.fy;
  x[0] = (((Real)u - (Real)f.cx)*ifx)*D;
  x[1] = (((Real)v - (Real)f.cy)*ify)*D;
  x[2] = D;
}

// --------------------------------------------------------------------------
// Per-pixel residuals and Jacobians, Eqs. (2)-(4).  With y = T x and the left
// perturbation exp(xi^) y ~ y + rho + phi x y, dS/drho = grad S and
// dS/dphi = y x grad S; likewise for the model intensity.
// --------------------------------------------------------------------------
template <class Real>
struct PixelTerms {
  bool ok = false;
  Real rd = 0, Jd[6] = {0};
  Real rc = 0, Jc[6] = {0};
};

template <class Real>
PixelTerms<Real> pixel_terms(const Map<Real>& m, const Real x[3], const double* T, Real I_pix) {
  PixelTerms<Real> pt;
  Real R[9], t[3], y[3];
  pose_split<Real>(T, R, t);
  transform(R, t, x, y);
  Sample<Real> s = sample_at(m, y);
  if (!s.ok) return pt;
  if (!(std::fabs(s.S) < (Real)m.P.truncation)) return pt;
  pt.rd = s.S;
  pt.rc = s.Iv - I_pix;
  const Real* g = s.gS;
  const Real* h = s.gI;
  Real cS[3] = {y[1]*g[2] - y[2]*g[1], y[2]*g[0] - y[0]*g[2], y[0]*g[1] - y[1]*g[0]};
  Real cI[3] = {y[1]*h[2] - y[2]*h[1], y[2]*h[0] - y[0]*h[2], y[0]*h[1] - y[1]*h[0]};
  for (int a = 0; a < 3; ++a) {
    pt.Jd[a] = g[a];
    pt.Jd[3+a] = cS[a];
    pt.Jc[a] = h[a];
    pt.Jc[3+a] = cI[a];
  }
  pt.ok = true;
  return pt;
}

// Normal equations of E = E_d + w_c E_c (Eq. 4) over the pixels of one pyramid
// level: H (21 upper-triangle terms, row-major), g (6), cost, count.
template <class Real>
void normal_equations(const Map<Real>& m, const Frame& f, const double* T, const uint8_t* mask,
                      int level, float w_c, double out[29]) {
  for (int i = 0; i < 29; ++i) out[i] = 0;
  const int step = 1 << level;
  const double wc = (double)w_c;
  // The sums run over each row of the level (rows are independent), then
  // over the rows in order, so the result does not depend on how rows are
  // shared out over threads in the OpenMP build.
  const int nv = (f.H + step - 1) / step;
  std::vector<std::array<double, 29>> rows((size_t)nv);
#pragma omp parallel for schedule(dynamic, 1)
  for (int iv = 0; iv < nv; ++iv) {
    const int v = iv*step;
    std::array<double, 29>& acc = rows[iv];
    acc.fill(0.0);
    for (int u = 0; u < f.W; u += step) {
      float D = depth_at(f, u, v);
      if (!depth_valid(D, m.P.depth_max)) continue;
      if (mask && mask[(size_t)v*f.W + u]) continue;
      Real x[3];
      backproject<Real>(f, u, v, (Real)D, x);
      Real I = luminance<Real>(f.rgb + 3*((size_t)v*f.W + u));
      PixelTerms<Real> pt = pixel_terms(m, x, T, I);
      if (!pt.ok) continue;
      int k = 0;
      for (int i = 0; i < 6; ++i)
        for (int j = i; j < 6; ++j) {
          acc[k++] += (double)pt.Jd[i]*(double)pt.Jd[j] + wc*((double)pt.Jc[i]*(double)pt.Jc[j]);
        }
      for (int i = 0; i < 6; ++i)
        acc[21+i] += (double)pt.Jd[i]*(double)pt.rd + wc*((double)pt.Jc[i]*(double)pt.rc);
      acc[27] += (double)pt.rd*(double)pt.rd + wc*((double)pt.rc*(double)pt.rc);
      acc[28] += 1.0;
    }
  }
  for (const std::array<double, 29>& acc : rows)
    for (int i = 0; i < 29; ++i) out[i] += acc[i];
}

// Solves (H + lambda diag H) delta = -g by Cholesky.  Returns false when a
// pivot is not above 1e-12 * trace(H).
bool solve6(const double* ne, double lambda, double delta[6]) {
  double A[6][6];
  int k = 0;
  for (int i = 0; i < 6; ++i)
    for (int j = i; j < 6; ++j) { A[i][j] = ne[k]; A[j][i] = ne[k]; ++k; }
  double tr = 0;
  for (int i = 0; i < 6; ++i) tr += A[i][i];
  for (int i = 0; i < 6; ++i) A[i][i] *= (1.0 + lambda);
  double L[6][6] = {{0}};
  for (int j = 0; j < 6; ++j) {
    double d = A[j][j];
    for (int p = 0; p < j; ++p) d -= L[j][p]*L[j][p];
    if (!(d > 1e-12*tr)) return false;
    L[j][j] = std::sqrt(d);
    for (int i = j + 1; i < 6; ++i) {
      double s = A[i][j];
      for (int p = 0; p < j; ++p) s -= L[i][p]*L[j][p];
      L[i][j] = s / L[j][j];
    }
  }
  double z[6];
  for (int i = 0; i < 6; ++i) {
    double s = -ne[21+i];
    for (int p = 0; p < i; ++p) s -= L[i][p]*z[p];
    z[i] = s / L[i][i];
  }
  for (int i = 5; i >= 0; --i) {
    double s = z[i];
    for (int p = i + 1; p < 6; ++p) s -= L[p][i]*delta[p];
    delta[i] = s / L[i][i];
  }
  return true;
}

// --------------------------------------------------------------------------
// Block-grid DDA (FP32).  Visits the cells of the segment q0 -> q1 (block
// units).  Cells: c = floor(q0) ... e = floor(q1).  Per axis the parameter
// of the next boundary is tmax = ((c + (step>0)) - q0) * (1/d) and grows by
// tdelta = step * (1/d).  Exactly |e-c|_1 steps are taken; each step moves
// the axis with the smallest tmax among those not yet at e (ties: x, y, z).
// --------------------------------------------------------------------------
template <class Visit>
void dda_cells(const float q0[3], const float q1[3], Visit visit) {
  int32_t c[3], e[3], step[3];
  float tmax[3], tdel[3];
  int64_t n = 0;
  for (int a = 0; a < 3; ++a) {
    c[a] = (int32_t)std::floor(q0[a]);
    e[a] = (int32_t)std::floor(q1[a]);
    float d = q1[a] - q0[a];
    step[a] = (e[a] > c[a]) ? 1 : ((e[a] < c[a]) ? -1 : 0);
    if (step[a] != 0) {
      float inv = 1.0f / d;
      float bound = (float)(c[a] + (step[a] > 0 ? 1 : 0));
      tmax[a] = (bound - q0[a])*inv;
      tdel[a] = (float)step[a]*inv;
    } else {
      tmax[a] = INFINITY;
      tdel[a] = INFINITY;
    }
    n += std::llabs((int64_t)e[a] - (int64_t)c[a]);
  }
  visit(c);
  for (int64_t k = 0; k < n; ++k) {
    int best = -1;
    for (int a = 0; a < 3; ++a) {
      if (c[a] == e[a]) continue;
      if (best < 0 || tmax[a] < tmax[best]) best = a;
    }
    c[best] += step[best];
    tmax[best] += tdel[best];
    visit(c);
  }
}

// Allocation: every block visited by the band (or carve) segment of every
// valid, unmasked pixel (Sections III-A, III-D).  Returns the visited set F.
void allocate(MapBase& m, const Frame& f, const double* T, const uint8_t* mask) {
  const Params& P = m.P;
  float R[9], t[3];
  pose_split<float>(T, R, t);
  const float ifx = 1.0f / f.fx, ify = 1.0f / f.fy;
  const float iB = 1.0f / (8.0f * P.voxel_size);
  const float tau = P.truncation;
  m.last_F.clear();
  m.F_set.clear();
  // The cells of every row's segments first (rows are independent), then
  // their insertion in pixel order, so the map and F come out the same
  // however the first loop is shared out over threads in the OpenMP build.
  std::vector<std::vector<Key>> cells((size_t)f.H);
#pragma omp parallel for schedule(dynamic, 1)
  for (int v = 0; v < f.H; ++v)
    for (int u = 0; u < f.W; ++u) {
      float D = depth_at(f, u, v);
      if (!(D > 0.0f)) continue;  // no measurement
      if (mask && mask[(size_t)v*f.W + u]) continue;
      bool carve = (u % P.carve_stride == 0) && (v % P.carve_stride == 0);
      // a measurement beyond depth_max is too far to be integrated but still
      // shows free space up to the clipping plane (Sec. III-D): only its carve
      // segment is walked, and it ends at the clipping plane
      bool far = !(D <= P.depth_max);
      if (far && !carve) continue;
      float zn = carve ? 0.0f : std::max(D - tau, 0.0f);
      float zf = far ? P.depth_max : D + tau;
      float rx = ((float)u - f.cx)*ifx, ry = ((float)v - f.cy)*ify;
      float X0[3] = {rx*zn, ry*zn, zn}, X1[3] = {rx*zf, ry*zf, zf};
      float P0[3], P1[3];
      transform(R, t, X0, P0);
      transform(R, t, X1, P1);
      float q0[3], q1[3];
      for (int a = 0; a < 3; ++a) { q0[a] = P0[a]*iB; q1[a] = P1[a]*iB; }
      dda_cells(q0, q1, [&](const int32_t* c) { cells[v].push_back(Key{c[0], c[1], c[2]}); });
    }
  for (const std::vector<Key>& row : cells)
    for (const Key& k : row) {
      m.add_block(k);
      if (m.F_set.insert(k).second) m.last_F.push_back(k);
    }
}

// Whole-block carving test of the compact free-space reading (FP32, in
// this order in the kernels too).  Depth cells: per 8x8 pixels, the
// smallest depth of the cell's measured pixels (D > 0, also beyond the
// clipping plane), or 0 when a pixel of the cell is masked or none is
// measured.  A block is carved whole when its 8 corner voxels, transformed
// as the integration transforms voxels, lie more than 1 mm in front of the
// camera and at least 1 mm before the clipping plane, the nearest pixels of
// their projections, widened by one pixel, span a rectangle inside the
// image covering at most 64 cells, and every one of those cells holds a
// depth more than tau + 1 mm beyond the block's farthest corner.  With every
// pixel measured and unmasked, the per-voxel rule would then carve every
// voxel of the block (the voxels' depths and pixels lie within the corners'
// range, far inside the margins); unmeasured pixels inside the rectangle
// are carved over.
constexpr int kCell = 8;

std::vector<float> depth_cells(const Frame& f, const uint8_t* mask, int& cw) {
  cw = (f.W + kCell - 1) / kCell;
  const int ch = (f.H + kCell - 1) / kCell;
  std::vector<float> cells((size_t)cw*ch);
  for (int cv = 0; cv < ch; ++cv)
    for (int cu = 0; cu < cw; ++cu) {
      float e = INFINITY;
      bool masked = false;
      for (int v = cv*kCell; v < std::min(cv*kCell + kCell, f.H); ++v)
        for (int u = cu*kCell; u < std::min(cu*kCell + kCell, f.W); ++u) {
          if (mask && mask[(size_t)v*f.W + u]) masked = true;
          float D = depth_at(f, u, v);
          if (D > 0.0f) e = std::min(e, D);
        }
      cells[(size_t)cv*cw + cu] = (masked || e == INFINITY) ? 0.0f : e;
    }
  return cells;
}

bool carve_whole(const Params& P, const Frame& f, const std::vector<float>& cells, int cw, const float R[9],
                 const float t[3], const Key& b) {
  const float s = P.voxel_size, margin = 1.0e-3f;
  float zmin = INFINITY, zmax = -INFINITY, umin = INFINITY, umax = -INFINITY, vmin = INFINITY, vmax = -INFINITY;
  for (int k = 0; k < 8; ++k) {
    int32_t vi[3] = {8*b.x + ((k & 1) ? 7 : 0), 8*b.y + ((k & 2) ? 7 : 0), 8*b.z + ((k & 4) ? 7 : 0)};
    float d[3], X[3];
    for (int a = 0; a < 3; ++a) d[a] = (float)vi[a]*s - t[a];
    for (int j = 0; j < 3; ++j) X[j] = (R[j]*d[0] + R[3+j]*d[1]) + R[6+j]*d[2];
    zmin = std::min(zmin, X[2]);
    zmax = std::max(zmax, X[2]);
    const float zz = std::max(X[2], margin);
    const float uf = f.fx*(X[0]/zz) + f.cx, vf = f.fy*(X[1]/zz) + f.cy;
    umin = std::min(umin, uf); umax = std::max(umax, uf);
    vmin = std::min(vmin, vf); vmax = std::max(vmax, vf);
  }
  if (!(zmin > margin && zmax + margin <= P.depth_max)) return false;
  const float u0 = std::floor(umin + 0.5f) - 1.0f, u1 = std::floor(umax + 0.5f) + 1.0f;
  const float v0 = std::floor(vmin + 0.5f) - 1.0f, v1 = std::floor(vmax + 0.5f) + 1.0f;
  if (!(u0 >= 0.0f && v0 >= 0.0f && u1 <= (float)(f.W - 1) && v1 <= (float)(f.H - 1))) return false;
  const int c0 = (int)u0 / kCell, c1 = (int)u1 / kCell, r0 = (int)v0 / kCell, r1 = (int)v1 / kCell;
  if ((c1 - c0 + 1)*(r1 - r0 + 1) > 64) return false;
  float dmin = INFINITY;
  for (int r = r0; r <= r1; ++r)
    for (int c = c0; c <= c1; ++c) dmin = std::min(dmin, cells[(size_t)r*cw + c]);
  return dmin > zmax + P.truncation + margin;
}

// The per-voxel rule's decision for voxel l of block b (FP32): 0 no update,
// 1 band update (d = eta, colour), 2 free-space update (d = tau); for an
// update, the pixel (u, v) and depth D it came from.
inline int voxel_kind(const Params& P, const Frame& f, const uint8_t* mask, const float Rf[9], const float tf[3],
                      const Key& b, int l, int& u, int& v, float& D) {
  const float s = P.voxel_size, tau = P.truncation, zclip = P.depth_max;
  int32_t vi[3] = {8*b.x + (l & 7), 8*b.y + ((l >> 3) & 7), 8*b.z + (l >> 6)};
  // X = R^T (v s - t)
  float d[3], X[3];
  for (int a = 0; a < 3; ++a) d[a] = (float)vi[a]*s - tf[a];
  for (int j = 0; j < 3; ++j) X[j] = (Rf[j]*d[0] + Rf[3+j]*d[1]) + Rf[6+j]*d[2];
  if (!(X[2] > 0.0f)) return 0;
  float uf = f.fx*(X[0]/X[2]) + f.cx;
  float vf = f.fy*(X[1]/X[2]) + f.cy;
  float ur = std::floor(uf + 0.5f), vr = std::floor(vf + 0.5f);
  if (!(ur >= 0.0f && ur < (float)f.W && vr >= 0.0f && vr < (float)f.H)) return 0;
  u = (int)ur;
  v = (int)vr;
  D = depth_at(f, u, v);
  if (!(D > 0.0f)) return 0;  // no measurement
  if (mask && mask[(size_t)v*f.W + u]) return 0;
  float eta = D - X[2];
  if (eta < -tau) return 0;  // behind the surface
  bool band = (eta <= tau);
  // the band of a measurement beyond depth_max is not integrated; the free
  // space in front of it is carved like any other (Sec. III-D)
  if (band && !(D <= P.depth_max)) return 0;
  if (!band && !(X[2] <= zclip)) return 0;
  return band ? 1 : 2;
}

// Integration (Sections III-A, III-C, III-D): running weighted average of the
// truncated projective distance, free space carved to tau, masked pixels
// ignored.  Decisions in FP32; values in Real.  counts: band updates, free
// updates, blocks carved whole (compact free space: free blocks counted
// once, their voxels not counted as updates).
template <class Real>
void integrate(Map<Real>& m, const Frame& f, const double* T, const uint8_t* mask, int64_t counts[3]) {
  const Params& P = m.P;
  float Rf[9], tf[3];
  pose_split<float>(T, Rf, tf);
  Real Rr[9], tr[3];
  pose_split<Real>(T, Rr, tr);
  const float s = P.voxel_size, tau = P.truncation, zclip = P.depth_max;
  counts[0] = counts[1] = counts[2] = 0;
  std::vector<Key> F = m.last_F;
  std::sort(F.begin(), F.end());
  // Compact free space: the whole-block test of every listed block.  A free
  // block carved whole only counts the frame.  Another free block is
  // evaluated voxel by voxel: if some voxel gets a band update it becomes a
  // block of voxels (starting from the free value) and takes the frame's
  // updates below; if every voxel is carved the frame counts for it; else
  // (some carved, some not updated) it is left as it is, so a free block's
  // value always stands for space observed free in all of its voxels.
  enum { kPerVoxel = 0, kWhole = 1, kDone = 2, kPending = 3 };
  std::vector<char> state(F.size(), kPerVoxel);
  int64_t n_whole = 0;
  if (P.free_blocks) {
    int cw = 0;
    const std::vector<float> cells = depth_cells(f, mask, cw);
    for (size_t bi = 0; bi < F.size(); ++bi) {
      const bool whole = carve_whole(P, f, cells, cw, Rf, tf, F[bi]);
      n_whole += whole;
      state[bi] = whole ? kWhole : kPerVoxel;
      auto it = m.free_blk.find(F[bi]);
      if (it == m.free_blk.end()) continue;
      if (whole) {
        Voxel<Real>& fv = it->second;
        fv.sdf = (Real)tau;
        fv.w = std::min(fv.w + (Real)1, (Real)P.max_weight);
        state[bi] = kDone;
      } else {
        state[bi] = kPending;
      }
    }
    // the pending free blocks' voxel decisions (independent of each other)
    std::vector<char> any_band(F.size(), 0), all_free(F.size(), 0);
#pragma omp parallel for schedule(dynamic, 16)
    for (size_t bi = 0; bi < F.size(); ++bi) {
      if (state[bi] != kPending) continue;
      bool band = false, all = true;
      for (int l = 0; l < 512; ++l) {
        int u, v;
        float D;
        const int k = voxel_kind(P, f, mask, Rf, tf, F[bi], l, u, v, D);
        band |= (k == 1);
        all &= (k == 2);
      }
      any_band[bi] = band;
      all_free[bi] = all;
    }
    for (size_t bi = 0; bi < F.size(); ++bi) {
      if (state[bi] != kPending) continue;
      auto it = m.free_blk.find(F[bi]);
      if (any_band[bi]) {
        m.blocks.emplace(F[bi], std::vector<Voxel<Real>>(512, it->second));
        m.free_blk.erase(it);
        state[bi] = kPerVoxel;
      } else {
        if (all_free[bi]) {
          it->second.sdf = (Real)tau;
          it->second.w = std::min(it->second.w + (Real)1, (Real)P.max_weight);
        }
        state[bi] = kDone;
      }
    }
  }
  // blocks are independent (each voxel is updated from its own value and the
  // frame), so the OpenMP build shares them out over threads
  int64_t n_band = 0, n_free = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : n_band, n_free)
  for (size_t bi = 0; bi < F.size(); ++bi) {
    const Key& b = F[bi];
    if (state[bi] == kDone) continue;  // a free block: counted, no voxels
    auto& blk = m.blocks.at(b);
    if (state[bi] == kWhole) {
      // carved whole: every voxel takes the free-space update
      for (int l = 0; l < 512; ++l) {
        Voxel<Real>& vx = blk[l];
        Real W = vx.w;
        vx.sdf = m.store_sdf((W*vx.sdf + (Real)tau) / (W + (Real)1));
        vx.w = std::min(W + (Real)1, (Real)P.max_weight);
      }
      n_free += 512;
      continue;
    }
    for (int l = 0; l < 512; ++l) {
      int u, v;
      float D;
      const int kind = voxel_kind(P, f, mask, Rf, tf, b, l, u, v, D);
      if (kind == 0) continue;
      const bool band = (kind == 1);
      // --- value path in Real
      Real dval;
      if (band) {
        int32_t vi[3] = {8*b.x + (l & 7), 8*b.y + ((l >> 3) & 7), 8*b.z + (l >> 6)};
        Real dr[3], Xz;
        for (int a = 0; a < 3; ++a) dr[a] = (Real)vi[a]*(Real)s - tr[a];
        Xz = (Rr[2]*dr[0] + Rr[5]*dr[1]) + Rr[8]*dr[2];
        dval = (Real)D - Xz;
      } else {
        dval = (Real)tau;
      }
      Voxel<Real>& vx = blk[l];
      Real W = vx.w;
      vx.sdf = m.store_sdf((W*vx.sdf + dval) / (W + (Real)1));
      if (band) {
        const uint8_t* c = f.rgb + 3*((size_t)v*f.W + u);
        for (int k = 0; k < 3; ++k) {
          Real cn = std::nearbyint((W*(Real)vx.rgb[k] + (Real)c[k]) / (W + (Real)1));
          vx.rgb[k] = (uint8_t)std::min((Real)255, std::max((Real)0, cn));
        }
        n_band++;
      } else {
        n_free++;
      }
      vx.w = std::min(W + (Real)1, (Real)P.max_weight);
    }
  }
  counts[0] = n_band;
  counts[1] = n_free;
  counts[2] = n_whole;
}

// Dynamics mask (Section III-C): r = S^2 at the registered pose (defined where
// the trilinear sample exists), raw = r > gamma tau^2, 3x3 erosion, depth-aware
// flood fill (Algorithm 1), 3x3 dilation.  All in FP32.
void floodfill(const uint8_t* seeds, const float* D, int W, int H, float theta, uint8_t* out) {
  // Algorithm 1 as a work queue: a pixel joins once, the first time some
  // member p has it as a neighbour with |D(p) - D(n)| < theta D(p).
  std::memcpy(out, seeds, (size_t)W*H);
  std::deque<int> Q;
  for (int i = 0; i < W*H; ++i)
    if (seeds[i]) Q.push_back(i);
  while (!Q.empty()) {
    int p = Q.front();
    Q.pop_front();
    int pu = p % W, pv = p / W;
    for (int dv = -1; dv <= 1; ++dv)
      for (int du = -1; du <= 1; ++du) {
        if (!du && !dv) continue;
        int nu = pu + du, nv = pv + dv;
        if (nu < 0 || nv < 0 || nu >= W || nv >= H) continue;
        int n = nv*W + nu;
        if (out[n]) continue;
        if (std::fabs(D[p] - D[n]) < theta*D[p]) {
          out[n] = 1;
          Q.push_back(n);
        }
      }
  }
}

void morph3x3(const uint8_t* in, int W, int H, bool erode, uint8_t* out) {
  for (int v = 0; v < H; ++v)
    for (int u = 0; u < W; ++u) {
      int all = 1, any = 0;
      for (int dv = -1; dv <= 1; ++dv)
        for (int du = -1; du <= 1; ++du) {
          int nu = u + du, nv = v + dv;
          int val = (nu >= 0 && nv >= 0 && nu < W && nv < H) ? in[nv*W + nu] : 0;
          all &= (val != 0);
          any |= (val != 0);
        }
      out[v*W + u] = (uint8_t)(erode ? all : any);
    }
}

void dynamic_mask(const Map<float>& m, const Frame& f, const double* T, float gamma, float theta,
                  uint8_t* raw, uint8_t* eroded, uint8_t* filled, uint8_t* final_, float* residual) {
  const int W = f.W, H = f.H;
  float R[9], t[3];
  pose_split<float>(T, R, t);
  const float tau = m.P.truncation;
  const float thr = gamma*(tau*tau);
  std::vector<float> Dff((size_t)W*H);
#pragma omp parallel for schedule(dynamic, 1)
  for (int v = 0; v < H; ++v)
    for (int u = 0; u < W; ++u) {
      size_t i = (size_t)v*W + u;
      float D = depth_at(f, u, v);
      bool ok = depth_valid(D, m.P.depth_max);
      Dff[i] = ok ? D : 0.0f;
      raw[i] = 0;
      if (residual) residual[i] = -1.0f;
      if (!ok) continue;
      float x[3], y[3];
      backproject<float>(f, u, v, D, x);
      transform(R, t, x, y);
      Sample<float> s = sample_at(m, y);
      if (!s.ok) continue;
      float r = s.S*s.S;
      if (residual) residual[i] = r;
      raw[i] = (r > thr) ? 1 : 0;
    }
  morph3x3(raw, W, H, true, eroded);
  floodfill(eroded, Dff.data(), W, H, theta, filled);
  morph3x3(filled, W, H, false, final_);
}

// Zero crossings of the SDF along voxel edges (the surface the mesh is cut
// from): voxels v and v+e with weight > 0, |sdf| < tau and opposite signs.
template <class Real>
int64_t surface(const Map<Real>& m, double* out, int64_t cap) {
  std::vector<Key> keys;
  for (auto& kv : m.blocks) keys.push_back(kv.first);
  std::sort(keys.begin(), keys.end());
  const Real s = (Real)m.P.voxel_size, tau = (Real)m.P.truncation;
  int64_t n = 0;
  for (const Key& b : keys) {
    const auto& blk = m.blocks.at(b);
    for (int l = 0; l < 512; ++l) {
      const Voxel<Real>& a = blk[l];
      if (!(a.w > 0) || !(std::fabs(a.sdf) < tau)) continue;
      int32_t vi[3] = {8*b.x + (l & 7), 8*b.y + ((l >> 3) & 7), 8*b.z + (l >> 6)};
      for (int ax = 0; ax < 3; ++ax) {
        int32_t nb[3] = {vi[0], vi[1], vi[2]};
        nb[ax] += 1;
        const Voxel<Real>* c = m.voxel(nb[0], nb[1], nb[2]);
        if (!c || !(c->w > 0) || !(std::fabs(c->sdf) < tau)) continue;
        if ((a.sdf > 0) == (c->sdf > 0)) continue;
        Real tt = a.sdf / (a.sdf - c->sdf);
        if (n < cap) {
          double* o = out + 7*n;
          for (int k = 0; k < 3; ++k) o[k] = (double)((Real)vi[k]*s);
          o[ax] = (double)((Real)vi[ax]*s + tt*s);
          o[3] = a.rgb[0]; o[4] = a.rgb[1]; o[5] = a.rgb[2];
          o[6] = ax;
        }
        ++n;
      }
    }
  }
  return n;
}

// Triangle mesh of the zero level set (the model is shown as a mesh, Sec. I
// and Fig. 1), by marching tetrahedra.  Reading: a cube of 8 voxel centres
// (lower corner v, corner k = dx + 2 dy + 4 dz at v + (dx, dy, dz)) is meshed
// when all 8 voxels exist, are observed (w > 0) and have |sdf| < tau (the
// condition the zero-crossing extraction applies per edge).  The cube is cut
// into the six tetrahedra along its diagonal 0-7, (0, a, a|b, 7) for the six
// orders of the axis bits a, b, c; neighbouring cubes cut their shared faces
// alike, so the mesh is closed wherever the cubes are.  Inside means
// sdf < 0.  A tetrahedron with one vertex on its own side gives one triangle
// (the crossings of that vertex's three edges), with two and two a quad (two
// triangles).  A crossing on edge (a, b), a the corner whose bits are a
// subset of b's, is P_a + t (P_b - P_a) with t = f_a / (f_a - f_b), per axis
// in the order written, so the same grid edge gives the same point in every
// tetrahedron and cube.  Triangles face the observed (positive) side: a
// triangle whose normal (q1 - q0) x (q2 - q0) has a negative dot product with
// (sum of outside vertices / their count - sum of inside vertices / their
// count), scaled to (n_in * sum_out - n_out * sum_in), is reversed.
// out: 9 values per triangle (3 vertices x, y, z); returns the count.
template <class Real>
int64_t mesh(const Map<Real>& m, double* out, int64_t cap) {
  static const int kTets[6][4] = {{0, 1, 3, 7}, {0, 1, 5, 7}, {0, 2, 3, 7},
                                  {0, 2, 6, 7}, {0, 4, 5, 7}, {0, 4, 6, 7}};
  std::vector<Key> keys;
  for (auto& kv : m.blocks) keys.push_back(kv.first);
  std::sort(keys.begin(), keys.end());
  const Real s = (Real)m.P.voxel_size, tau = (Real)m.P.truncation;
  int64_t n = 0;
  auto emit = [&](const Real* q0, const Real* q1, const Real* q2) {
    if (n < cap) {
      double* o = out + 9*n;
      for (int a = 0; a < 3; ++a) { o[a] = (double)q0[a]; o[3+a] = (double)q1[a]; o[6+a] = (double)q2[a]; }
    }
    ++n;
  };
  for (const Key& b : keys) {
    for (int l = 0; l < 512; ++l) {
      const int32_t v[3] = {8*b.x + (l & 7), 8*b.y + ((l >> 3) & 7), 8*b.z + (l >> 6)};
      Real f[8], P[8][3];
      bool ok = true;
      for (int k = 0; k < 8 && ok; ++k) {
        const int32_t c[3] = {v[0] + (k & 1), v[1] + ((k >> 1) & 1), v[2] + (k >> 2)};
        const Voxel<Real>* vx = m.voxel(c[0], c[1], c[2]);
        if (!vx || !(vx->w > 0) || !(std::fabs(vx->sdf) < tau)) { ok = false; break; }
        f[k] = vx->sdf;
        for (int a = 0; a < 3; ++a) P[k][a] = (Real)c[a] * s;
      }
      if (!ok) continue;
      for (const auto& T : kTets) {
        int ins[4], outs[4], ni = 0, no = 0;
        for (int j = 0; j < 4; ++j) {
          if (f[T[j]] < 0) ins[ni++] = T[j];
          else outs[no++] = T[j];
        }
        if (ni == 0 || no == 0) continue;
        // crossing point of the edge between corners i and o
        auto cross = [&](int i, int o, Real* q) {
          const int lo = (i & o) == i ? i : o, hi = lo == i ? o : i;  // lo's bits are a subset of hi's
          const Real t = f[lo] / (f[lo] - f[hi]);
          for (int a = 0; a < 3; ++a) q[a] = P[lo][a] + t * (P[hi][a] - P[lo][a]);
        };
        // orientation reference: n_in * sum(outside) - n_out * sum(inside)
        Real ref[3];
        for (int a = 0; a < 3; ++a) {
          Real so = 0, si = 0;
          for (int j = 0; j < no; ++j) so += P[outs[j]][a];
          for (int j = 0; j < ni; ++j) si += P[ins[j]][a];
          ref[a] = (Real)ni * so - (Real)no * si;
        }
        auto facing = [&](const Real* q0, const Real* q1, const Real* q2) {
          const Real e1[3] = {q1[0] - q0[0], q1[1] - q0[1], q1[2] - q0[2]};
          const Real e2[3] = {q2[0] - q0[0], q2[1] - q0[1], q2[2] - q0[2]};
          const Real nx = e1[1]*e2[2] - e1[2]*e2[1], ny = e1[2]*e2[0] - e1[0]*e2[2], nz = e1[0]*e2[1] - e1[1]*e2[0];
          return (nx*ref[0] + ny*ref[1]) + nz*ref[2] >= 0;
        };
        if (ni == 1 || no == 1) {
          const int lone = ni == 1 ? ins[0] : outs[0];
          const int* other = ni == 1 ? outs : ins;
          Real q[3][3];
          for (int j = 0; j < 3; ++j) cross(lone, other[j], q[j]);
          if (facing(q[0], q[1], q[2])) emit(q[0], q[1], q[2]);
          else emit(q[0], q[2], q[1]);
        } else {
          // quad: (i0,o0) (i0,o1) (i1,o1) (i1,o0) is a cycle of crossing edges
          Real q[4][3];
          cross(ins[0], outs[0], q[0]);
          cross(ins[0], outs[1], q[1]);
          cross(ins[1], outs[1], q[2]);
          cross(ins[1], outs[0], q[3]);
          if (facing(q[0], q[1], q[2])) {
            emit(q[0], q[1], q[2]);
            emit(q[0], q[2], q[3]);
          } else {
            emit(q[0], q[2], q[1]);
            emit(q[0], q[3], q[2]);
          }
        }
      }
    }
  }
  return n;
}

// Virtual depth (Sec. III-E, second option for invalid measurements): a
// model of the last n frames is ray cast from a frame's registered pose and
// the zeros of the frame's depth are replaced by the virtual depth, the
// pixels the model does not explain by a far value.  Reading: along pixel
// (u, v)'s ray the samples are taken at camera depths z_k = z_near + k step,
// step = tau / 2 (so the band |sdf| < tau holds at least three samples), for
// z_k <= z_far, at the back-projection of (u, v) at depth z_k (Eq. 1); the
// virtual depth is the first crossing from a defined sample S_{k-1} > 0 to a
// defined sample S_k <= 0, z_{k-1} + step (S_{k-1} / (S_{k-1} - S_k)); 0 if
// there is none.  With only_invalid, pixels whose raw depth is not zero keep
// their depth (metres) and the zeros get the virtual depth or far_value;
// otherwise every pixel gets its virtual depth (0 without a crossing).
template <class Real>
void raycast(const Map<Real>& m, const Frame& f, const double* T, Real z_near, Real z_far, Real far_value,
             bool only_invalid, float* out) {
  Real R[9], t[3];
  pose_split<Real>(T, R, t);
  const Real step = (Real)0.5 * (Real)m.P.truncation;
  for (int v = 0; v < f.H; ++v)
    for (int u = 0; u < f.W; ++u) {
      const float D = depth_at(f, u, v);
      float& o = out[(size_t)v*f.W + u];
      if (only_invalid && D != 0.0f) { o = D; continue; }
      Real hit = 0, prev = 0;
      bool have_prev = false;
      for (int k = 0;; ++k) {
        const Real z = z_near + (Real)k * step;
        if (!(z <= z_far)) break;
        Real x[3], y[3];
        backproject<Real>(f, u, v, z, x);
        transform(R, t, x, y);
        Sample<Real> sm = sample_at(m, y);
        if (!sm.ok) { have_prev = false; continue; }
        if (have_prev && prev > 0 && sm.S <= 0) {
          const Real zp = z_near + (Real)(k - 1) * step;
          hit = zp + step * (prev / (prev - sm.S));
          break;
        }
        prev = sm.S;
        have_prev = true;
      }
      o = only_invalid ? (hit > 0 ? (float)hit : (float)far_value) : (float)hit;
    }
}

template <class Real>
Map<Real>* as(void* h) { return static_cast<Map<Real>*>(static_cast<MapBase*>(h)); }


}  // namespace

// ============================================================================
// C interface (host pointers only).  Handles are MapBase*; real_bits says
// which template instantiation sits behind it.
// ============================================================================
extern "C" {

typedef struct {
  int32_t width, height;
  float fx, fy, cx, cy;
  const void* depth;
  int32_t depth_u16;
  float depth_scale;
  const uint8_t* rgb;
} orc_frame;

struct OrcMap {
  int real_bits;
  MapBase* m;
};

static Frame to_frame(const orc_frame* f) {
  Frame r;
  r.W = f->width; r.H = f->height;
  r.fx = f->fx; r.fy = f->fy; r.cx = f->cx; r.cy = f->cy;
  r.depth = f->depth; r.depth_u16 = f->depth_u16; r.depth_scale = f->depth_scale;
  r.rgb = f->rgb;
  return r;
}

void* orc_map_new(int real_bits, int storage, float voxel_size, float truncation, float depth_max,
                  int max_weight, int carve_stride, int free_blocks) {
  OrcMap* h = new OrcMap;
  h->real_bits = real_bits;
  if (real_bits == 32) h->m = new Map<float>();
  else h->m = new Map<double>();
  h->m->P = Params{voxel_size, truncation, depth_max, max_weight, carve_stride, storage, free_blocks};
  return h;
}

void orc_map_free(void* p) {
  OrcMap* h = (OrcMap*)p;
  delete h->m;
  delete h;
}

int64_t orc_map_num_blocks(void* p) { return ((OrcMap*)p)->m->num_blocks(); }

// Blocks that hold voxels (all blocks unless the map keeps free space compact).
int64_t orc_map_num_voxel_blocks(void* p) { return ((OrcMap*)p)->m->num_voxel_blocks(); }

// Allocation; returns |F| and writes F's keys (sorted) if out_keys != NULL.
int64_t orc_allocate(void* p, const orc_frame* fr, const double* T, const uint8_t* mask,
                     int32_t* out_keys, int64_t cap) {
  OrcMap* h = (OrcMap*)p;
  allocate(*h->m, to_frame(fr), T, mask);
  std::vector<Key> F = h->m->last_F;
  std::sort(F.begin(), F.end());
  if (out_keys)
    for (int64_t i = 0; i < (int64_t)F.size() && i < cap; ++i) {
      out_keys[3*i] = F[i].x; out_keys[3*i+1] = F[i].y; out_keys[3*i+2] = F[i].z;
    }
  return (int64_t)F.size();
}

int orc_integrate(void* p, const orc_frame* fr, const double* T, const uint8_t* mask, int64_t* counts) {
  OrcMap* h = (OrcMap*)p;
  int64_t c[3];
  if (h->real_bits == 32) integrate(*as<float>(h->m), to_frame(fr), T, mask, c);
  else integrate(*as<double>(h->m), to_frame(fr), T, mask, c);
  if (counts) { counts[0] = c[0]; counts[1] = c[1]; counts[2] = c[2]; }
  return 0;
}

int orc_normal_equations(void* p, const orc_frame* fr, const double* T, const uint8_t* mask, int level,
                         float w_c, double* out29) {
  OrcMap* h = (OrcMap*)p;
  if (h->real_bits == 32) normal_equations(*as<float>(h->m), to_frame(fr), T, mask, level, w_c, out29);
  else normal_equations(*as<double>(h->m), to_frame(fr), T, mask, level, w_c, out29);
  return 0;
}

// Coarse-to-fine Gauss-Newton / LM tracking (Section III-B).  stats (nullable,
// 4+levels doubles): final cost, final count, iterations done, flags
// (1 = too few pixels, 2 = singular system), then per-level pixel counts of
// each level's first iteration.
int orc_track(void* p, const orc_frame* fr, double* T, const uint8_t* mask, int levels, int iters,
              float w_c, int min_valid, double lm_lambda, double* stats) {
  OrcMap* h = (OrcMap*)p;
  Frame f = to_frame(fr);
  double ne[29] = {0};
  int done = 0, flags = 0;
  std::vector<double> first(levels, 0.0);
  for (int l = levels - 1; l >= 0 && !flags; --l) {
    for (int it = 0; it < iters; ++it) {
      if (h->real_bits == 32) normal_equations(*as<float>(h->m), f, T, mask, l, w_c, ne);
      else normal_equations(*as<double>(h->m), f, T, mask, l, w_c, ne);
      if (it == 0) first[l] = ne[28];
      if (ne[28] < min_valid) { flags |= 1; break; }
      double delta[6];
      if (!solve6(ne, lm_lambda, delta)) { flags |= 2; break; }
      pose_left_update(delta, T);
      ++done;
    }
  }
  if (stats) {
    stats[0] = ne[27]; stats[1] = ne[28]; stats[2] = done; stats[3] = flags;
    for (int l = 0; l < levels; ++l) stats[4+l] = first[l];
  }
  return flags;
}

// Levenberg-Marquardt variant of the same coarse-to-fine registration (the
// solver Section III-B names), as a fixed budget of cost evaluations:
// evaluation e (e = 0 .. levels*iters - 1, level by level) computes the normal
// equations at the candidate pose C_e.  The first evaluation of each level is
// accepted as it is (its cost is not comparable with the previous level's);
// later ones are accepted when they have at least min_valid residuals and a
// mean cost (cost / count) no larger than the accepted one's; then lambda is
// divided by 10, and a rejected candidate multiplies it by 10 (at least 1e-4).
// Unless e is the last evaluation, the next candidate is exp(delta^) T_a with
// (H_a + lambda diag H_a) delta = -g_a from the accepted pose T_a and its
// normal equations.  The result is the accepted pose after the last decision.
// stats as orc_track, with stats[2] = accepted steps.  trace (nullable,
// 5 doubles per evaluation): level, cost/count of C_e, count, accepted (0/1),
// lambda after the decision.
int orc_track_lm(void* p, const orc_frame* fr, double* T, const uint8_t* mask, int levels, int iters,
                 float w_c, int min_valid, double lambda0, double* stats, double* trace) {
  OrcMap* h = (OrcMap*)p;
  Frame f = to_frame(fr);
  double ne_c[29] = {0}, ne_a[29] = {0};
  double Ta[16], C[16];
  for (int i = 0; i < 16; ++i) Ta[i] = C[i] = T[i];
  double lambda = lambda0;
  int done = 0, flags = 0, e = 0;
  const int total = levels * iters;
  std::vector<double> first(levels, 0.0);
  for (int l = levels - 1; l >= 0 && !flags; --l) {
    for (int it = 0; it < iters; ++it, ++e) {
      if (h->real_bits == 32) normal_equations(*as<float>(h->m), f, C, mask, l, w_c, ne_c);
      else normal_equations(*as<double>(h->m), f, C, mask, l, w_c, ne_c);
      bool accept;
      if (it == 0) {
        first[l] = ne_c[28];
        accept = true;
      } else {
        accept = ne_c[28] >= min_valid && ne_c[27] / ne_c[28] <= ne_a[27] / ne_a[28];
        lambda = accept ? lambda / 10.0 : std::max(lambda * 10.0, 1e-4);
        if (accept) ++done;
      }
      if (accept) {
        for (int i = 0; i < 29; ++i) ne_a[i] = ne_c[i];
        for (int i = 0; i < 16; ++i) Ta[i] = C[i];
      }
      if (trace) {
        double* t = trace + 5 * e;
        t[0] = l; t[1] = ne_c[28] > 0 ? ne_c[27] / ne_c[28] : 0.0; t[2] = ne_c[28]; t[3] = accept; t[4] = lambda;
      }
      if (e == total - 1) break;
      if (ne_a[28] < min_valid) { flags |= 1; break; }
      double delta[6];
      if (!solve6(ne_a, lambda, delta)) { flags |= 2; break; }
      for (int i = 0; i < 16; ++i) C[i] = Ta[i];
      pose_left_update(delta, C);
    }
  }
  for (int i = 0; i < 16; ++i) T[i] = Ta[i];
  if (stats) {
    stats[0] = ne_a[27]; stats[1] = ne_a[28]; stats[2] = done; stats[3] = flags;
    for (int l = 0; l < levels; ++l) stats[4+l] = first[l];
  }
  return flags;
}

int orc_mask(void* p, const orc_frame* fr, const double* T, float gamma, float theta, uint8_t* raw,
             uint8_t* eroded, uint8_t* filled, uint8_t* final_, float* residual) {
  OrcMap* h = (OrcMap*)p;
  if (h->real_bits != 32) return -1;  // the mask is a decision: FP32 only
  dynamic_mask(*as<float>(h->m), to_frame(fr), T, gamma, theta, raw, eroded, filled, final_, residual);
  return 0;
}

// Sorted export: keys (n x 3), sdf and weight (n x 512, as double), rgb
// (n x 512 x 3).  Returns the number of blocks (writes at most cap).
int64_t orc_export(void* p, int32_t* keys, double* sdf, double* w, uint8_t* rgb, int64_t cap) {
  OrcMap* h = (OrcMap*)p;
  auto dump = [&](auto* m) -> int64_t {
    std::vector<Key> ks;
    for (auto& kv : m->blocks) ks.push_back(kv.first);
    std::sort(ks.begin(), ks.end());
    for (int64_t i = 0; i < (int64_t)ks.size() && i < cap; ++i) {
      const auto& blk = m->blocks.at(ks[i]);
      if (keys) { keys[3*i] = ks[i].x; keys[3*i+1] = ks[i].y; keys[3*i+2] = ks[i].z; }
      for (int l = 0; l < 512; ++l) {
        if (sdf) sdf[512*i + l] = (double)blk[l].sdf;
        if (w) w[512*i + l] = (double)blk[l].w;
        if (rgb) for (int k = 0; k < 3; ++k) rgb[3*(512*i + l) + k] = blk[l].rgb[k];
      }
    }
    return (int64_t)ks.size();
  };
  if (h->real_bits == 32) return dump(as<float>(h->m));
  return dump(as<double>(h->m));
}

// Free blocks (compact free space): keys (sorted) and the weight their voxels
// read as.  Returns the count.
int64_t orc_export_free(void* p, int32_t* keys, double* w, int64_t cap) {
  OrcMap* h = (OrcMap*)p;
  auto dump = [&](auto* m) -> int64_t {
    std::vector<Key> ks;
    for (auto& kv : m->free_blk) ks.push_back(kv.first);
    std::sort(ks.begin(), ks.end());
    for (int64_t i = 0; i < (int64_t)ks.size() && i < cap; ++i) {
      if (keys) { keys[3*i] = ks[i].x; keys[3*i+1] = ks[i].y; keys[3*i+2] = ks[i].z; }
      if (w) w[i] = (double)m->free_blk.at(ks[i]).w;
    }
    return (int64_t)ks.size();
  };
  if (h->real_bits == 32) return dump(as<float>(h->m));
  return dump(as<double>(h->m));
}

int orc_import(void* p, const int32_t* keys, const double* sdf, const double* w, const uint8_t* rgb,
               int64_t n) {
  OrcMap* h = (OrcMap*)p;
  auto load = [&](auto* m) {
    using V = typename std::remove_reference<decltype(m->blocks.begin()->second[0])>::type;
    for (int64_t i = 0; i < n; ++i) {
      Key k{keys[3*i], keys[3*i+1], keys[3*i+2]};
      std::vector<V> blk(512);
      for (int l = 0; l < 512; ++l) {
        blk[l].sdf = (decltype(blk[l].sdf))sdf[512*i + l];
        blk[l].w = (decltype(blk[l].w))w[512*i + l];
        for (int c = 0; c < 3; ++c) blk[l].rgb[c] = rgb[3*(512*i + l) + c];
      }
      m->blocks[k] = blk;
    }
  };
  if (h->real_bits == 32) load(as<float>(h->m));
  else load(as<double>(h->m));
  return 0;
}

// Surface points: 7 doubles each (x, y, z, r, g, b, axis).  Returns the count.
int64_t orc_surface(void* p, double* out, int64_t cap) {
  OrcMap* h = (OrcMap*)p;
  if (h->real_bits == 32) return surface(*as<float>(h->m), out, cap);
  return surface(*as<double>(h->m), out, cap);
}

// Virtual depth / filled depth of a frame (float32 metres, W*H).
int orc_raycast(void* p, const orc_frame* fr, const double* T, double z_near, double z_far, double far_value,
                int only_invalid, float* out) {
  OrcMap* h = (OrcMap*)p;
  if (h->real_bits == 32)
    raycast(*as<float>(h->m), to_frame(fr), T, (float)z_near, (float)z_far, (float)far_value, only_invalid != 0, out);
  else
    raycast(*as<double>(h->m), to_frame(fr), T, (double)(float)z_near, (double)(float)z_far, (double)(float)far_value,
            only_invalid != 0, out);
  return 0;
}

// Mesh triangles: 9 doubles each.  Returns the count (writes at most cap).
int64_t orc_mesh(void* p, double* out, int64_t cap) {
  OrcMap* h = (OrcMap*)p;
  if (h->real_bits == 32) return mesh(*as<float>(h->m), out, cap);
  return mesh(*as<double>(h->m), out, cap);
}

// ---- single-operation entry points used by the pins ----------------------
void orc_se3_exp(const double* xi, double* T) { se3_exp(xi, T); }
void orc_pose_left_update(const double* xi, double* T) { pose_left_update(xi, T); }
int orc_solve6(const double* ne, double lambda, double* delta) { return solve6(ne, lambda, delta) ? 0 : 1; }
float orc_round_to_half(float x) { return round_to_half(x); }

// Sample (S, dS/dy[3], Iv, dIv/dy[3]) at world point y; returns 1 if defined.
int orc_sample(void* p, const double* y, double* out8) {
  OrcMap* h = (OrcMap*)p;
  auto go = [&](auto* m, auto zero) {
    using Real = decltype(zero);
    Real yy[3] = {(Real)y[0], (Real)y[1], (Real)y[2]};
    Sample<Real> s = sample_at(*m, yy);
    out8[0] = s.S;
    for (int a = 0; a < 3; ++a) { out8[1+a] = s.gS[a]; out8[5+a] = s.gI[a]; }
    out8[4] = s.Iv;
    return s.ok ? 1 : 0;
  };
  if (h->real_bits == 32) return go(as<float>(h->m), 0.0f);
  return go(as<double>(h->m), 0.0);
}

// Residuals and Jacobians of one camera point x under pose T (14 doubles:
// r_d, J_d[6], r_c, J_c[6]); returns 1 if the pixel is used.
int orc_pixel_terms(void* p, const double* x, const double* T, double I_pix, double* out14) {
  OrcMap* h = (OrcMap*)p;
  auto go = [&](auto* m, auto zero) {
    using Real = decltype(zero);
    Real xx[3] = {(Real)x[0], (Real)x[1], (Real)x[2]};
    PixelTerms<Real> t = pixel_terms(*m, xx, T, (Real)I_pix);
    out14[0] = t.rd;
    out14[7] = t.rc;
    for (int a = 0; a < 6; ++a) { out14[1+a] = t.Jd[a]; out14[8+a] = t.Jc[a]; }
    return t.ok ? 1 : 0;
  };
  if (h->real_bits == 32) return go(as<float>(h->m), 0.0f);
  return go(as<double>(h->m), 0.0);
}

// DDA cells of one segment (block units); returns the count, writes <= cap.
int64_t orc_dda(const float* q0, const float* q1, int32_t* out, int64_t cap) {
  int64_t n = 0;
  dda_cells(q0, q1, [&](const int32_t* c) {
    if (n < cap) { out[3*n] = c[0]; out[3*n+1] = c[1]; out[3*n+2] = c[2]; }
    ++n;
  });
  return n;
}

void orc_floodfill(const uint8_t* seeds, const float* D, int W, int H, float theta, uint8_t* out) {
  floodfill(seeds, D, W, H, theta, out);
}

void orc_morph3x3(const uint8_t* in, int W, int H, int erode, uint8_t* out) {
  morph3x3(in, W, H, erode != 0, out);
}

// Threads of the OpenMP build (the plain build runs one thread and ignores
// the request).
void orc_set_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
