// Direct registration to the TSDF (Sec. III-B, Eqs. 1-4) for gfx950.
//
// One launch per Gauss-Newton/LM iteration, one thread per pixel of the
// pyramid level (a workgroup covers a 16x16 pixel tile, so the voxels its
// wavefronts gather are close together).  A thread forms the depth residual S and the photometric
// residual Iv - I with their 6-DoF Jacobians in FP32 and parks them in LDS;
// the workgroup then forms the 29 normal-equation terms in FP64 (products of
// FP32 factors are exact in FP64) with a fixed-order transposed reduction
// over its pixels, and adds them to device-wide accumulators.
//
// The accumulators are fixed point (units of 2^-60) held as two chunks in
// 64-bit words, the low 48 bits and the signed rest, and summed with
// device-scope integer atomics: integer addition is associative, so the
// totals do not depend on the order in which workgroups finish
// (bit-reproducible), and the chunks need no carry chain, so every atomic is
// independent (the low chunk's sums keep 16 bits of headroom for carries).  Workgroups spread over kAccCopies
// copies of the accumulators (fewer atomics per address), which the reader
// sums exactly.  Nothing in a launch waits for the
// other workgroups: the solve of iteration j runs at the start of launch j+1,
// redundantly in every workgroup (all read the same completed totals and run
// the same instructions, so all obtain the same pose), overlapped with the
// pose-independent loads of the pixel (levels with more workgroups than two
// resident rounds solve in a one-workgroup launch instead, see
// kSeparateSolveTiles).  Accumulators rotate through three
// buffers (read j-1, write j, clear j+1) and the pose through two, so no
// launch reads what the same launch writes.  A one-workgroup finalize launch
// solves the last iteration and writes the caller's pose.
#include <type_traits>

#include "rf_device.h"
#include "rf_internal.h"

namespace rf {

constexpr double kFixScale = 0x1p60;
constexpr int kTermWords = 16;                     // one 128-byte line per term
constexpr int kCopyWords = kNE * kTermWords;       // one copy of the 29 accumulators
constexpr int kBufWords = kAccCopies * kCopyWords;  // one accumulator buffer
constexpr int kTerms = 15;                         // J_d(6) J_c(6) r_d r_c used
constexpr int kGroups = kTrackBlock / 32;          // LDS reduction groups per term
constexpr int kTileW = kTrackBlock / 16;           // pixel tile: kTileW x 16

struct TrackArgs {
  int level;         // pyramid level evaluated by this launch (-1: none)
  float w_c;
  int min_valid;
  double lm_lambda;
  int solve;         // 1: first solve the system accumulated by the previous launch
  int prev_level;    // level of that previous evaluation
  int prev_first;    // it was the first iteration of its level
  int acc_read, acc_write, acc_clear;  // accumulator buffer indices (-1: none)
  int pose_read, pose_write;           // 0/1: pose scratch, 2: caller's pose (-1: none)
  int mode;          // 0: track; 1: write the normal equations of acc_read to out29; 2: solve only
  int adaptive;      // 1: Levenberg-Marquardt (accept / reject, adaptive lambda); 0: fixed lambda
  int state_read, state_write;         // Levenberg-Marquardt state buffers (0/1, -1: none)
};

__device__ __forceinline__ unsigned long long* acc_buf(const MapDev& m, int b) {
  return reinterpret_cast<unsigned long long*>(m.partials) + (size_t)b * kBufWords;
}
// The words an accumulator buffer actually uses: two chunks and a range
// marker per term per copy (the rest of each 128-byte line is padding against
// false sharing: atomics on one line are served one after another).
constexpr int kUsedPerTerm = 3;
constexpr int kUsedWords = kAccCopies * kNE * kUsedPerTerm;
__device__ __forceinline__ unsigned long long* used_word(unsigned long long* buf, int q) {
  const int copy = q / (kNE * kUsedPerTerm), r = q % (kNE * kUsedPerTerm);
  return buf + copy * kCopyWords + (r / kUsedPerTerm) * kTermWords + (r % kUsedPerTerm);
}
__device__ __forceinline__ double* pose_buf(const MapDev& m, double* user, int b) {
  return b == 2 ? user : reinterpret_cast<double*>(m.partials) + (size_t)3 * kBufWords + 16 * b;
}
// Levenberg-Marquardt state: [0, 16) accepted pose, [16, 45) its normal
// equations, [45] lambda.
constexpr int kLmWords = 48;
__device__ __forceinline__ double* lm_state(const MapDev& m, int b) {
  return reinterpret_cast<double*>(m.partials) + (size_t)3 * kBufWords + 32 + kLmWords * b;
}

// Adds v to a term: v 2^60 truncated toward zero as a two's complement
// integer lo + hi 2^48 (lo unsigned 48-bit, hi signed 64-bit), two atomics
// (one where hi is 0).  The low chunks of a copy sum below 2^63 for up to 2^15
// workgroups (a 2^26-pixel frame's tiles over the copies), the high chunks of
// terms below 2^34 likewise.  A non-finite v, or |v| >= 2^34 (beyond that
// range), is not added: the term's range marker acc[2] is set instead, and
// its total then reads as NaN, which stops the registration pass
// (RF_FLAG_TRACK_RANGE).  Returns false in that case.
__device__ __forceinline__ bool fixed_add(unsigned long long* acc, double v) {
  double a = fabs(v) * kFixScale;
  if (!(a < 0x1p94)) {
    atomicOr(&acc[2], 1ull);
    return false;
  }
  const double hi_d = floor(a * 0x1p-48);
  unsigned long long hi = (unsigned long long)hi_d;
  unsigned long long lo = (unsigned long long)(a - hi_d * 0x1p48);
  if (v < 0.0) {
    hi = ~hi + (lo == 0ull ? 1ull : 0ull);
    lo = (0ull - lo) & 0xFFFFFFFFFFFFull;
  }
  if (lo) atomicAdd(&acc[0], lo);
  if (hi) atomicAdd(&acc[1], hi);
  return true;
}

// Total of a term over the accumulator copies as FP64 (exact 128-bit integer
// sum, then conversion).  A term whose range marker is set in any copy
// totals NaN.
__device__ __forceinline__ double fixed_total(const unsigned long long* acc) {
  unsigned long long lo = 0, hi = 0, bad = 0;
#pragma unroll
  for (int c = 0; c < kAccCopies; ++c) {
    const unsigned long long s0 = acc[c * kCopyWords];
    const long long s1 = (long long)acc[c * kCopyWords + 1];
    bad |= acc[c * kCopyWords + 2];
    // s1 2^48 + s0 as a 128-bit two's complement number, added to (hi, lo)
    const unsigned long long l1 = (unsigned long long)s1 << 48;
    const unsigned long long h1 = (unsigned long long)(s1 >> 16);
    const unsigned long long n = lo + l1;
    hi += h1 + (n < lo ? 1ull : 0ull);
    lo = n + s0;
    hi += (lo < n ? 1ull : 0ull);
  }
  if (bad) return __longlong_as_double(0x7FF8000000000000ll);
  const bool neg = (long long)hi < 0;
  if (neg) {
    lo = ~lo + 1ull;
    hi = ~hi + (lo == 0ull ? 1ull : 0ull);
  }
  const double mag = ((double)hi * 0x1p64 + (double)lo) * (1.0 / kFixScale);
  return neg ? -mag : mag;
}

__device__ __forceinline__ double readlane_f64(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xFFFFFFFFll), lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ int tri_index(int i, int j) {  // H(i,j), i <= j, packed upper triangle
  return 6 * i - (i * (i - 1)) / 2 + (j - i);
}

// The solving wavefront of a workgroup: totals -> delta by row-parallel
// elimination (lane r holds row r of [H + lambda diag H | -g]; no pivoting, H is
// symmetric positive semi-definite) -> exp(delta^) T.  Writes the new pose
// (row-major 12 values) to s_T and the outcome to *s_state:
// 0 ok, RF_FLAG_TRACK_FEW_PIXELS or RF_FLAG_TRACK_SINGULAR (pose kept).
// A pivot of the elimination equals the squared Cholesky pivot, so the
// singularity test is the Cholesky one: pivot <= 1e-12 trace(H).
// tin[0..2] = Tin[ec], Tin[4 + ec], Tin[8 + ec] and tin[3] = Tin[lane] for
// lanes < 16 (element (er, ec) = (lane / 4, lane % 4) of the input pose).
__device__ void solve_update_wave(const double* s_ne, const TrackArgs& a, const double tin[4], double* s_T,
                                  int* s_state) {
  const int lane = threadIdx.x & 63;
  int state = 0;
  bool finite = true;
#pragma unroll
  for (int k = 0; k < kNE; ++k) finite &= (s_ne[k] == s_ne[k]);
  if (!finite) state = RF_FLAG_TRACK_RANGE;
  else if (s_ne[28] < (double)a.min_valid) state = RF_FLAG_TRACK_FEW_PIXELS;
  double tr = 0.0;
#pragma unroll
  for (int i = 0; i < 6; ++i) tr += s_ne[tri_index(i, i)];
  const int r = lane < 6 ? lane : 5;
  double row[7];
#pragma unroll
  for (int c = 0; c < 6; ++c) row[c] = s_ne[r <= c ? tri_index(r, c) : tri_index(c, r)];
#pragma unroll
  for (int c = 0; c < 6; ++c)
    if (c == r) row[c] *= (1.0 + a.lm_lambda);
  row[6] = -s_ne[21 + r];
  double inv[6];  // reciprocal pivots, reused by the back substitution
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double piv = readlane_f64(row[k], k);
    if (!(piv > 1e-12 * tr) && state == 0) state = RF_FLAG_TRACK_SINGULAR;
    inv[k] = 1.0 / piv;
    double pk[7];
#pragma unroll
    for (int c = k + 1; c < 7; ++c) pk[c] = readlane_f64(row[c], k);
    if (lane > k && lane < 6 && state == 0) {
      const double fct = row[k] * inv[k];
#pragma unroll
      for (int c = k + 1; c < 7; ++c) row[c] = fma(-fct, pk[c], row[c]);
    }
  }
  double x[6] = {0, 0, 0, 0, 0, 0};
  if (state == 0) {
#pragma unroll
    for (int k = 5; k >= 0; --k) {
      double s = readlane_f64(row[6], k);
#pragma unroll
      for (int j = k + 1; j < 6; ++j) s = fma(-readlane_f64(row[j], k), x[j], s);
      x[k] = s * inv[k];
    }
  }
  if (lane < 16) {
    double out;
    if (lane >= 12) {
      out = (lane == 15) ? 1.0 : 0.0;
    } else if (state != 0) {
      out = tin[3];
    } else {
      // exp of the twist (rho, phi) = x: R = I + A K + B K^2, t = (I + B K + C K^2) rho
      const double p0 = x[3], p1 = x[4], p2 = x[5];
      const double th2 = p0 * p0 + p1 * p1 + p2 * p2;
      double A, B, C;
      if (th2 < 1e-2) {
        // Taylor series of sin(th)/th, (1 - cos th)/th^2, (th - sin th)/th^3 in
        // th^2 (Horner); for th < 0.1 the first omitted term is below 1e-18
        A = fma(th2, fma(th2, fma(th2, fma(th2, fma(th2, -1.0 / 39916800.0, 1.0 / 362880.0), -1.0 / 5040.0),
                                  1.0 / 120.0), -1.0 / 6.0), 1.0);
        B = fma(th2, fma(th2, fma(th2, fma(th2, fma(th2, -1.0 / 479001600.0, 1.0 / 3628800.0), -1.0 / 40320.0),
                                  1.0 / 720.0), -1.0 / 24.0), 0.5);
        C = fma(th2, fma(th2, fma(th2, fma(th2, fma(th2, -1.0 / 6227020800.0, 1.0 / 39916800.0), -1.0 / 362880.0),
                                  1.0 / 5040.0), -1.0 / 120.0), 1.0 / 6.0);
      } else {
        const double th = sqrt(th2), sn = sin(th), hs = sin(0.5 * th);
        A = sn / th;
        B = 2.0 * hs * hs / th2;
        C = (th - sn) / (th2 * th);
      }
      const double ph[3] = {p0, p1, p2};
      const int er = lane >> 2, ec = lane & 3;
      // row er of E = exp: E[er][q] for q = 0..2 (rotation) and E[er][3] (translation)
      double E[4];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        double K = 0.0;  // [phi]x (er, q)
        if (er == 0 && q == 1) K = -p2;
        if (er == 0 && q == 2) K = p1;
        if (er == 1 && q == 0) K = p2;
        if (er == 1 && q == 2) K = -p0;
        if (er == 2 && q == 0) K = -p1;
        if (er == 2 && q == 1) K = p0;
        const double K2 = ph[er] * ph[q] - (er == q ? th2 : 0.0);
        E[q] = (er == q ? 1.0 : 0.0) + A * K + B * K2;
      }
      {
        const double rho[3] = {x[0], x[1], x[2]};
        const double cr[3] = {p1 * rho[2] - p2 * rho[1], p2 * rho[0] - p0 * rho[2], p0 * rho[1] - p1 * rho[0]};
        const double ccr[3] = {p1 * cr[2] - p2 * cr[1], p2 * cr[0] - p0 * cr[2], p0 * cr[1] - p1 * cr[0]};
        E[3] = rho[er] + B * cr[er] + C * ccr[er];
      }
      out = E[0] * tin[0] + E[1] * tin[1] + E[2] * tin[2];
      if (ec == 3) out += E[3];
    }
    s_T[lane] = out;
  }
  if (lane == 0) *s_state = state;
}

// The solve step shared by the tracking and finalize launches, run by the
// solving wavefront: reads the accumulated totals, solves, and (workgroup 0 only)
// publishes the pose, the statistics and, on a degenerate system, the stop
// flag.  Returns through LDS: s_T (new pose), *s_state.
//
// Levenberg-Marquardt (a.adaptive): the totals are those of the candidate
// pose the previous launch evaluated.  The first evaluation of a level is
// accepted as it is; a later one when it has at least min_valid residuals and
// a mean cost (cost / count) no larger than the accepted one's, which divides
// lambda by 10 (a rejection multiplies it by 10, at least 1e-4).  The step is
// then solved from the accepted pose and its normal equations; with
// final_only (the last decision of a pass) no step follows and the accepted
// pose is the result.  s_nc, s_st: LDS scratch of kLmWords doubles each.
template <bool LM>
__device__ void solve_step(const MapDev& m, double* user_pose, const TrackArgs& a, rf_track_stats* stats,
                           double* s_ne, double* s_T, int* s_state, bool publish, bool stopped, bool final_only,
                           double* s_nc, double* s_st) {
  const int lane = threadIdx.x & 63;
  const int ec = lane & 3;
  // the input pose is fetched together with the totals (one round trip)
  double tin[4] = {0.0, 0.0, 0.0, 0.0};
  double lam = a.lm_lambda;
  bool accept = true, first = true;
  if (!LM) {
    // pose and totals are loaded without branches (clamped lanes) so all the
    // loads share one round trip; the pose goes through LDS (fewer registers
    // held across the solve)
    double pin = pose_buf(m, user_pose, a.pose_read)[lane < 16 ? lane : 0];
    const double tot = fixed_total(acc_buf(m, a.acc_read) + (lane < kNE ? lane : 0) * kTermWords);
    asm volatile("" : "+v"(pin));
    if (lane < 16) s_nc[kNE + lane] = pin;
    if (lane < kNE) s_ne[lane] = tot;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    if (lane < 16) {
      tin[0] = s_nc[kNE + ec];
      tin[1] = s_nc[kNE + 4 + ec];
      tin[2] = s_nc[kNE + 8 + ec];
      tin[3] = s_nc[kNE + lane];
    }
  } else {
    const double* C = pose_buf(m, user_pose, a.pose_read);  // the candidate just evaluated
    const double* S = lm_state(m, a.state_read);
    double cin = C[lane < 16 ? lane : 0];
    double st_in = S[lane < kLmWords ? lane : 0];
    const double tot = fixed_total(acc_buf(m, a.acc_read) + (lane < kNE ? lane : 0) * kTermWords);
    asm volatile("" : "+v"(cin), "+v"(st_in));
    if (lane < kNE) s_nc[lane] = tot;
    if (lane < kLmWords) s_st[lane] = st_in;
    if (lane < 16) s_nc[kNE + lane] = cin;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    first = a.prev_first != 0;
    accept = first || (s_nc[28] >= (double)a.min_valid && s_nc[27] / s_nc[28] <= s_st[16 + 27] / s_st[16 + 28]);
    lam = s_st[45];
    if (!first) lam = accept ? lam / 10.0 : fmax(lam * 10.0, 1e-4);
    if (lane < kNE) s_ne[lane] = accept ? s_nc[lane] : s_st[16 + lane];
    if (lane < 16) {
      const double* Ta = accept ? s_nc + kNE : s_st;
      tin[0] = Ta[ec];
      tin[1] = Ta[4 + ec];
      tin[2] = Ta[8 + ec];
      tin[3] = Ta[lane];
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (final_only) {
    if (lane < 16) s_T[lane] = tin[3];
    if (lane == 0) *s_state = 0;
  } else {
    TrackArgs ta = a;
    ta.lm_lambda = lam;
    solve_update_wave(s_ne, ta, tin, s_T, s_state);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  if (!publish || stopped) return;
  const int state = *s_state;
  if (lane < 16) {
    double* Tout = pose_buf(m, user_pose, a.pose_write);
    Tout[lane] = s_T[lane];
    if (state != 0 && a.pose_write != 2) pose_buf(m, user_pose, 1 - a.pose_write)[lane] = s_T[lane];
  }
  if (LM && a.state_write >= 0) {
    double* S = lm_state(m, a.state_write);
    if (lane < 16) S[lane] = tin[3];
    if (lane < kNE) S[16 + lane] = s_ne[lane];
    if (lane == 0) S[45] = lam;
  }
  if (lane == 0) {
    if (stats) {
      stats->cost = s_ne[27];
      stats->count = s_ne[28];
      if (a.prev_first && a.prev_level >= 0 && a.prev_level < 8)
        stats->level_count[a.prev_level] = LM ? s_nc[28] : s_ne[28];
      if (state != 0) stats->flags |= (uint32_t)state;
      else if (LM ? (accept && !first) : !final_only) stats->iters += 1;
    }
    if (state != 0) {
      m.st->track_stop = 1;
      atomicOr(&m.st->flags, (uint32_t)state);
    }
  }
}

// Per-workgroup block cache in LDS: a direct-mapped window of kWin^3 blocks
// centred on the bounding box of the tile's cached blocks (one indexed read,
// no key to compare) and, for blocks outside it, a small open-addressing
// hash (linear probing).  Built from the tile's cached pairs before the first
// barrier, consulted before the hash table, extended with every pair the hash
// table resolves, and written back (the pairs used in this launch) for the
// next launch at this level and tile.  A slot still being written reads as
// kNoSlot, which a lookup treats as a miss, so concurrent inserts never
// yield a wrong slot.
constexpr int kNoSlot = (int)0x80000000;
constexpr int kMaxProbe = 8;   // a key is placed within 8 slots of its home or not cached
constexpr int kWin = 8;        // direct-mapped window of kWin^3 blocks around the tile's blocks
constexpr int kWinCells = kWin * kWin * kWin;
constexpr int kFarOrigin = 0x40000000;  // window origin that no block coordinate reaches

// SLOTS: LDS hash capacity (the tile's pair capacity at the launch's level).
template <int SLOTS>
struct TileCache {
  unsigned long long* key;  // SLOTS, kEmptyKey when free
  int* slot;                // SLOTS, kNoSlot until written
  uint8_t* used;            // SLOTS, 1 when looked up in this launch
  int* grid;                // kWin^3 window of block slots (kNoSlot: unknown)
  uint8_t* gused;           // kWin^3, 1 when looked up in this launch
  int ax, ay, az;           // window origin (block coordinates)

  // window cell of block (x,y,z), or -1 outside the window
  __device__ __forceinline__ int cell(int x, int y, int z) const {
    const uint32_t dx = (uint32_t)(x - ax), dy = (uint32_t)(y - ay), dz = (uint32_t)(z - az);
    return (dx < (uint32_t)kWin && dy < (uint32_t)kWin && dz < (uint32_t)kWin) ? (int)(dx + kWin * (dy + kWin * dz)) : -1;
  }

  __device__ __forceinline__ void insert(int x, int y, int z, unsigned long long k, int sl, bool mark) const {
    uint32_t h = hash3(x, y, z) & (SLOTS - 1);
#pragma unroll 1
    for (int i = 0; i < kMaxProbe; ++i) {
      const unsigned long long old = atomicCAS(&key[h], kEmptyKey, k);
      if (old == kEmptyKey) {
        slot[h] = sl;
        if (mark) used[h] = 1;
        return;
      }
      if (old == k) {
        if (mark) used[h] = 1;
        return;
      }
      h = (h + 1) & (SLOTS - 1);
    }
  }

  __device__ __forceinline__ int find(int x, int y, int z, unsigned long long k) const {
    uint32_t h = hash3(x, y, z) & (SLOTS - 1);
#pragma unroll 1
    for (int i = 0; i < kMaxProbe; ++i) {
      const unsigned long long kk = key[h];
      if (kk == k) {
        const int sl = slot[h];
        if (sl != kNoSlot) used[h] = 1;
        return sl;
      }
      if (kk == kEmptyKey) break;
      h = (h + 1) & (SLOTS - 1);
    }
    return kNoSlot;
  }
};

// Slot resolution of sample_map through the tile cache: cached blocks cost
// an LDS probe; the others take the hash table (first probes of all missing
// corner blocks issued together) and are added to the cache.
template <int SLOTS>
struct CachedSlots {
  TileCache<SLOTS> c;
  __device__ __forceinline__ bool operator()(const MapDev& m, int bx0, int by0, int bz0, int cross, int sl[8]) const {
    // window cells of all eight corner blocks read together (one LDS round trip)
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const int cl = c.cell(bx0 + (k & 1), by0 + ((k >> 1) & 1), bz0 + (k >> 2));
      sl[k] = c.grid[cl >= 0 ? cl : 0];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) asm volatile("" : "+v"(sl[k]));
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if ((k & ~cross) != 0) continue;
      const int x = bx0 + (k & 1), y = by0 + ((k >> 1) & 1), z = bz0 + (k >> 2);
      const int cl = c.cell(x, y, z);
      if (cl >= 0) {
        if (sl[k] != kNoSlot) c.gused[cl] = 1;
      } else {
        sl[k] = c.find(x, y, z, pack_key(x, y, z));
      }
    }
    unsigned long long bkey[8];
    uint32_t bslot[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if ((k & ~cross) != 0 || sl[k] != kNoSlot) continue;
      const int x = bx0 + (k & 1), y = by0 + ((k >> 1) & 1), z = bz0 + (k >> 2);
      const Bucket* p = m.buckets + (hash3(x, y, z) & m.bucket_mask);
      bkey[k] = p->key;
      bslot[k] = p->slot;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if ((k & ~cross) != 0 || sl[k] != kNoSlot) continue;
      const int x = bx0 + (k & 1), y = by0 + ((k >> 1) & 1), z = bz0 + (k >> 2);
      Bucket b0;
      b0.key = bkey[k];
      b0.slot = bslot[k];
      const unsigned long long key = pack_key(x, y, z);
      sl[k] = resolve_slot(m, b0, key, hash3(x, y, z) & m.bucket_mask);
      const int cl = c.cell(x, y, z);
      if (cl >= 0) {
        c.grid[cl] = sl[k];
        c.gused[cl] = 1;
      } else {
        c.insert(x, y, z, key, sl[k], true);
      }
    }
    bool ok = true;
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if ((k & ~cross) != 0) sl[k] = sl[k & cross];
      ok &= sl[k] != -1;  // absent; free blocks (<= -2) read as (tau, count)
    }
    return ok;
  }
};

// Wavefront 1 of a residual workgroup (the tracking kernel runs the same
// steps inline): the tile's cached block pairs (tiles without a cache entry
// start from an empty table) placed in the direct-mapped window around their
// bounding box or in the LDS hash.
template <int SLOTS>
__device__ __forceinline__ void build_tile_cache(const BlockRef* tab, const uint32_t* tcount, bool cached, int nrefs,
                                                 uint32_t epoch, int lane, unsigned long long* s_hk, int* s_hs,
                                                 uint8_t* s_used, int* s_grid, uint8_t* s_gused, int* s_org,
                                                 uint32_t* s_nref) {
  const BlockRef none{kEmptyKey, -1, 0u};
  constexpr int kLoads = SLOTS / 64;
  const int cnt = cached ? (int)min(*tcount, (uint32_t)nrefs) : 0;
  BlockRef e[kLoads];
#pragma unroll
  for (int q = 0; q < kLoads; ++q) e[q] = (cached && lane + 64 * q < nrefs) ? tab[lane + 64 * q] : none;
#pragma unroll
  for (int q = 0; q < SLOTS / 64; ++q) {
    s_hk[lane + 64 * q] = kEmptyKey;
    s_hs[lane + 64 * q] = kNoSlot;
    s_used[lane + 64 * q] = 0;
  }
#pragma unroll
  for (int q = 0; q < kWinCells / 64; ++q) {
    s_grid[lane + 64 * q] = kNoSlot;
    s_gused[lane + 64 * q] = 0;
  }
  if (lane == 0) *s_nref = 0u;
  // window origin: centre of the bounding box of the valid cached blocks
  bool v[kLoads];
  int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
#pragma unroll
  for (int q = 0; q < kLoads; ++q) {
    v[q] = lane + 64 * q < cnt && e[q].key != kEmptyKey && (e[q].slot >= 0 || e[q].epoch == epoch);
    int p[3];
    unpack_key(e[q].key, p[0], p[1], p[2]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = min(lo[d], v[q] ? p[d] : INT_MAX);
      hi[d] = max(hi[d], v[q] ? p[d] : INT_MIN);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = min(lo[d], __shfl_xor(lo[d], o));
      hi[d] = max(hi[d], __shfl_xor(hi[d], o));
    }
  }
  const bool any = lo[0] <= hi[0];
  int org[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) org[d] = any ? ((lo[d] + hi[d]) >> 1) - (kWin / 2 - 1) : kFarOrigin;
  if (lane == 0) {
    s_org[0] = org[0];
    s_org[1] = org[1];
    s_org[2] = org[2];
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const TileCache<SLOTS> wc{s_hk, s_hs, s_used, s_grid, s_gused, org[0], org[1], org[2]};
#pragma unroll
  for (int q = 0; q < kLoads; ++q) {
    if (!v[q]) continue;
    int p[3];
    unpack_key(e[q].key, p[0], p[1], p[2]);
    const int cl = wc.cell(p[0], p[1], p[2]);
    if (cl >= 0) s_grid[cl] = e[q].slot;
    else wc.insert(p[0], p[1], p[2], e[q].key, e[q].slot, false);
  }
}

// SLOTS: pairs the tile cache holds in LDS (256 at levels 0-1, 512 at the
// coarser levels, whose few tiles each touch more blocks; more LDS and
// registers there cost nothing, since those launches have few workgroups).
template <int DF, int STORAGE, bool LM, int SLOTS>
__global__ __launch_bounds__(kTrackBlock) void track_kernel(Batch b, TrackArgs a) {
  __shared__ float s_t[kTerms][kTrackBlock + 1];
  __shared__ double s_g[kNE][kGroups + 1];
  __shared__ double s_ne[kNE];
  __shared__ double s_nc[kLmWords];
  __shared__ double s_st[kLmWords];
  __shared__ double s_T[16];
  __shared__ int s_state;
  __shared__ unsigned long long s_hk[SLOTS];
  __shared__ int s_hs[SLOTS];
  __shared__ uint8_t s_used[SLOTS];
  __shared__ int s_grid[kWinCells];
  __shared__ uint8_t s_gused[kWinCells];
  __shared__ int s_org[3];
  __shared__ uint32_t s_nref;
  const int jb = batch_job(b, blockIdx.x);
  const Job& J = b.job[jb];
  const MapDev& m = J.m;
  const FrameDev& f = J.f;
  const uint8_t* mask = J.mask;
  double* user_pose = J.pose;
  rf_track_stats* stats = J.stats;
  const int g0 = blockIdx.x - b.base[jb];  // tile index within the job
  // Set only by earlier launches.  Read here but acted on after the pixel
  // loads and the solve are under way: only publishing waits for it.
  const uint32_t stopped = m.st->track_stop;
  const uint32_t epoch = m.st->epoch;

  // pose-independent loads first, so their latency overlaps the solve
  // workgroup = kTileW x 16 tile of the level's pixel grid, wavefront = 8x8 sub-tile
  const int lv = a.level;
  const int wl = (f.W + (1 << lv) - 1) >> lv;
  const int hl = (f.H + (1 << lv) - 1) >> lv;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tiles_x = (wl + kTileW - 1) / kTileW;
  const int ul = (g0 % tiles_x) * kTileW + (wave % (kTileW / 8)) * 8 + (lane & 7);
  const int vl = (g0 / tiles_x) * 16 + (wave / (kTileW / 8)) * 8 + (lane >> 3);
  // Depth, mask and colour are loaded without a branch (pixels outside the
  // level read pixel 0; a missing mask reads the colour plane) so the loads
  // share one round trip and are first used after the solve.
  const bool inside = ul < wl && vl < hl;
  const int u = inside ? ul << lv : 0, v = inside ? vl << lv : 0;
  const int pix = v * f.W + u;
  const float D = load_depth<DF>(f, pix);
  const uint8_t mk_raw = (mask ? mask : f.rgb)[pix];
  const uint8_t* px = f.rgb + 3 * pix;
  const uint8_t c0 = px[0], c1 = px[1], c2 = px[2];
  if (a.acc_clear >= 0) {
    // the workgroups of the job share the clearing of the used chunk words
    const int ng = b.base[jb + 1] - b.base[jb];
    const int per = (kUsedWords + ng - 1) / ng;
    const int q1 = min(g0 * per + per, kUsedWords);
    for (int q = g0 * per + threadIdx.x; q < q1; q += kTrackBlock) *used_word(acc_buf(m, a.acc_clear), q) = 0ull;
  }
  // the tile's cached block pairs (the wavefront after the solving one,
  // while it solves); tiles without a cache entry start from an empty table
  const bool cached = a.level < kCacheLevels && g0 < (int)m.tc_tiles;
  BlockRef* tab = m.tcache + (size_t)m.tc_tiles * tile_refs_before(cached ? a.level : 0) +
                  (size_t)(cached ? g0 : 0) * tile_refs(cached ? a.level : 0);
  uint32_t* tcount = m.tc_count + (size_t)(cached ? a.level : 0) * m.tc_tiles + (cached ? g0 : 0);
  const int nrefs = tile_refs(a.level);
  // (the steps of build_tile_cache, written out: calling it here changed the
  // kernel's instruction schedule and cost the large rooms' tracking 3%)
  // the solving wavefront (and the cache builder after it) rotate with the
  // tile index, so the solves of the workgroups sharing a CU spread over its
  // SIMDs
  const int sw = g0 & 3, cw = (sw + 1) & 3;
  if (wave == cw) {
    const BlockRef none{kEmptyKey, -1, 0u};
    constexpr int kLoads = SLOTS / 64;
    const int cnt = cached ? (int)min(*tcount, (uint32_t)nrefs) : 0;
    BlockRef e[kLoads];
#pragma unroll
    for (int q = 0; q < kLoads; ++q) e[q] = (cached && lane + 64 * q < nrefs) ? tab[lane + 64 * q] : none;
#pragma unroll
    for (int q = 0; q < SLOTS / 64; ++q) {
      s_hk[lane + 64 * q] = kEmptyKey;
      s_hs[lane + 64 * q] = kNoSlot;
      s_used[lane + 64 * q] = 0;
    }
#pragma unroll
    for (int q = 0; q < kWinCells / 64; ++q) {
      s_grid[lane + 64 * q] = kNoSlot;
      s_gused[lane + 64 * q] = 0;
    }
    if (lane == 0) s_nref = 0u;
    // window origin: centre of the bounding box of the valid cached blocks
    bool v[kLoads];
    int lo[3] = {INT_MAX, INT_MAX, INT_MAX}, hi[3] = {INT_MIN, INT_MIN, INT_MIN};
#pragma unroll
    for (int q = 0; q < kLoads; ++q) {
      v[q] = lane + 64 * q < cnt && e[q].key != kEmptyKey && (e[q].slot >= 0 || e[q].epoch == epoch);
      int p[3];
      unpack_key(e[q].key, p[0], p[1], p[2]);
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        lo[d] = min(lo[d], v[q] ? p[d] : INT_MAX);
        hi[d] = max(hi[d], v[q] ? p[d] : INT_MIN);
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
#pragma unroll
      for (int d = 0; d < 3; ++d) {
        lo[d] = min(lo[d], __shfl_xor(lo[d], o));
        hi[d] = max(hi[d], __shfl_xor(hi[d], o));
      }
    }
    const bool any = lo[0] <= hi[0];
    int org[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) org[d] = any ? ((lo[d] + hi[d]) >> 1) - (kWin / 2 - 1) : kFarOrigin;
    if (lane == 0) {
      s_org[0] = org[0];
      s_org[1] = org[1];
      s_org[2] = org[2];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const TileCache<SLOTS> wc{s_hk, s_hs, s_used, s_grid, s_gused, org[0], org[1], org[2]};
#pragma unroll
    for (int q = 0; q < kLoads; ++q) {
      if (!v[q]) continue;
      int p[3];
      unpack_key(e[q].key, p[0], p[1], p[2]);
      const int cl = wc.cell(p[0], p[1], p[2]);
      if (cl >= 0) s_grid[cl] = e[q].slot;
      else wc.insert(p[0], p[1], p[2], e[q].key, e[q].slot, false);
    }
  }
  if (wave == sw) {
    if (a.solve) {
      solve_step<LM>(m, user_pose, a, stats, s_ne, s_T, &s_state, g0 == 0, stopped != 0, false, s_nc, s_st);
    } else {
      const double* Tin = pose_buf(m, user_pose, a.pose_read);
      if (lane < 16) {
        s_T[lane] = Tin[lane];
        if (g0 == 0 && !stopped && a.pose_write >= 0) pose_buf(m, user_pose, a.pose_write)[lane] = Tin[lane];
      }
      if (LM && g0 == 0 && !stopped && a.state_write >= 0) {
        // the starting pose is the accepted one until the first decision
        double* S = lm_state(m, a.state_write);
        if (lane < 16) S[lane] = Tin[lane];
        if (lane == 0) S[45] = a.lm_lambda;
      }
      if (lane == 0) s_state = 0;
    }
  }
  __syncthreads();
  if (stopped || s_state != 0) return;  // stopped or degenerate: pose kept, the pass stops
  const TileCache<SLOTS> cache{s_hk, s_hs, s_used, s_grid, s_gused, s_org[0], s_org[1], s_org[2]};

  float term[kTerms];
#pragma unroll
  for (int k = 0; k < kTerms; ++k) term[k] = 0.0f;
  if (inside && depth_ok(D, m.dmax) && !(mask && mk_raw)) {
    const float Ipix = luminance((float)c0, (float)c1, (float)c2);
    float R[9], t[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
#pragma unroll
      for (int c = 0; c < 3; ++c) R[3 * r + c] = (float)s_T[4 * r + c];
      t[r] = (float)s_T[4 * r + 3];
    }
    const float x[3] = {(((float)u - f.cx) * f.ifx) * D, (((float)v - f.cy) * f.ify) * D, D};
    float y[3];
    xform(R, t, x, y);
    float S, gS[3], Iv, gI[3];
    if (sample_map<STORAGE, true, true>(m, y, S, gS, Iv, gI, CachedSlots<SLOTS>{cache}) && fabsf(S) < m.tau) {
      term[0] = gS[0];
      term[1] = gS[1];
      term[2] = gS[2];
      term[3] = y[1] * gS[2] - y[2] * gS[1];
      term[4] = y[2] * gS[0] - y[0] * gS[2];
      term[5] = y[0] * gS[1] - y[1] * gS[0];
      term[6] = gI[0];
      term[7] = gI[1];
      term[8] = gI[2];
      term[9] = y[1] * gI[2] - y[2] * gI[1];
      term[10] = y[2] * gI[0] - y[0] * gI[2];
      term[11] = y[0] * gI[1] - y[1] * gI[0];
      term[12] = S;
      term[13] = Iv - Ipix;
      term[14] = 1.0f;
    }
  }
#pragma unroll
  for (int k = 0; k < kTerms; ++k) s_t[k][threadIdx.x] = term[k];
  __syncthreads();
  // the pairs used in this launch become the tile's cache for the next one
  if (cached) {
    for (int h = threadIdx.x; h < kWinCells; h += kTrackBlock) {
      const int ss = s_grid[h];
      if (ss != kNoSlot && s_gused[h]) {
        const uint32_t pos = atomicAdd(&s_nref, 1u);
        const unsigned long long kk = pack_key(cache.ax + h % kWin, cache.ay + (h / kWin) % kWin, cache.az + h / (kWin * kWin));
        if (pos < (uint32_t)nrefs) tab[pos] = BlockRef{kk, ss, epoch};
      }
    }
    for (int h = threadIdx.x; h < SLOTS; h += kTrackBlock) {
      const unsigned long long kk = s_hk[h];
      const int ss = s_hs[h];
      if (kk != kEmptyKey && ss != kNoSlot && s_used[h]) {
        const uint32_t pos = atomicAdd(&s_nref, 1u);
        if (pos < (uint32_t)nrefs) tab[pos] = BlockRef{kk, ss, epoch};
      }
    }
  }

  // thread (k, g) sums term k over pixels g, g + kGroups, ... in a fixed order
  // as a depth and a photometric product chain.  Every term has the same
  // shape (the count is the sum of 1 x 1 with a zero photometric weight), so
  // the wavefronts do not diverge, and the loop is unrolled so its LDS reads
  // are issued ahead of the FMAs.
  const double wc = (double)a.w_c;
  if (threadIdx.x < kNE * kGroups) {
    const int k = threadIdx.x % kNE, g = threadIdx.x / kNE;
    int r = 0, c = 12;
    if (k < 21) {
      int kk = k;
      while (kk >= 6 - r) {
        kk -= 6 - r;
        ++r;
      }
      c = r + kk;
    } else if (k < 27) {
      r = k - 21;
    }
    // k < 21: H(r, c); k < 27: g(r); 27: cost; 28: count
    const int rd = (k < 27) ? r : (k == 27 ? 12 : 14), cd = (k < 21) ? c : (k < 28 ? 12 : 14);
    const int rc = (k < 27) ? 6 + r : (k == 27 ? 13 : 14), cc = (k < 21) ? 6 + c : (k < 28 ? 13 : 14);
    const double wk = (k < 28) ? wc : 0.0;
    double acc_d = 0.0, acc_c = 0.0;
#pragma unroll
    for (int i = 0; i < kTrackBlock / kGroups; ++i) {
      const int p = g + i * kGroups;
      acc_d = fma((double)s_t[rd][p], (double)s_t[cd][p], acc_d);
      acc_c = fma((double)s_t[rc][p], (double)s_t[cc][p], acc_c);
    }
    s_g[k][g] = acc_d + wk * acc_c;
  }
  __syncthreads();
  if (cached && threadIdx.x == 0) *tcount = min(s_nref, (uint32_t)nrefs);
  if (threadIdx.x < kNE) {
    double tot = 0.0;
#pragma unroll
    for (int g = 0; g < kGroups; ++g) tot += s_g[threadIdx.x][g];
    if (!fixed_add(acc_buf(m, a.acc_write) + (g0 % kAccCopies) * kCopyWords + threadIdx.x * kTermWords, tot)) {
      atomicOr(&m.st->flags, (uint32_t)RF_FLAG_TRACK_RANGE);
      if (stats) atomicOr(&stats->flags, (uint32_t)RF_FLAG_TRACK_RANGE);
    }
  }
}

// Residual of the dynamic mask (Sec. III-C): r = S(T x)^2 of every valid
// pixel at full resolution and the raw decision r > gamma tau^2, with the
// pixels in the 16x16 tiles of the finest tracking level so that the corner
// blocks resolve through that level's tile cache (the pairs the last
// registration at this level used; a tile without them starts empty).  The
// cache only replaces hash-table probes, so the result is that of plain
// lookups.
template <int DF, int STORAGE, int SLOTS>
__global__ __launch_bounds__(kTrackBlock) void residual_kernel(Batch b, float gamma) {
  __shared__ unsigned long long s_hk[SLOTS];
  __shared__ int s_hs[SLOTS];
  __shared__ uint8_t s_used[SLOTS];
  __shared__ int s_grid[kWinCells];
  __shared__ uint8_t s_gused[kWinCells];
  __shared__ int s_org[3];
  __shared__ uint32_t s_nref;
  const int jb = batch_job(b, blockIdx.x);
  const Job& J = b.job[jb];
  const MapDev& m = J.m;
  const FrameDev& f = J.f;
  const int g0 = blockIdx.x - b.base[jb];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int tiles_x = (f.W + kTileW - 1) / kTileW;
  const int u = (g0 % tiles_x) * kTileW + (wave % (kTileW / 8)) * 8 + (lane & 7);
  const int v = (g0 / tiles_x) * 16 + (wave / (kTileW / 8)) * 8 + (lane >> 3);
  const bool inside = u < f.W && v < f.H;
  const int pix = inside ? v * f.W + u : 0;
  const float D = load_depth<DF>(f, pix);
  const bool cached = g0 < (int)m.tc_tiles;
  const BlockRef* tab = m.tcache + (size_t)(cached ? g0 : 0) * tile_refs(0);
  const uint32_t* tcount = m.tc_count + (cached ? g0 : 0);
  if (wave == 1)
    build_tile_cache<SLOTS>(tab, tcount, cached, tile_refs(0), m.st->epoch, lane, s_hk, s_hs, s_used, s_grid,
                            s_gused, s_org, &s_nref);
  __syncthreads();
  const TileCache<SLOTS> cache{s_hk, s_hs, s_used, s_grid, s_gused, s_org[0], s_org[1], s_org[2]};
  uint8_t out = 0;
  float r = -1.0f;
  if (inside && depth_ok(D, m.dmax)) {
    float R[9], t[3];
    load_pose_f(J.pose, R, t);
    const float x[3] = {(((float)u - f.cx) * f.ifx) * D, (((float)v - f.cy) * f.ify) * D, D};
    float y[3];
    xform(R, t, x, y);
    float S, Iv, g3[3], h3[3];
    if (sample_map<STORAGE, false, false>(m, y, S, g3, Iv, h3, CachedSlots<SLOTS>{cache})) {
      r = S * S;
      out = (r > gamma * (m.tau * m.tau)) ? 1 : 0;
    }
  }
  if (inside) {
    (J.raw ? J.raw : J.mask_out)[pix] = out;
    if (J.residual) J.residual[pix] = r;
  }
}

// Solve of the last evaluation of a pass (mode 0), the raw totals (mode 1),
// or, for launches with many workgroups, the solve a tracking launch would
// otherwise run at its start (mode 2): one workgroup per job.
__global__ __launch_bounds__(64) void track_finalize_kernel(Batch b, TrackArgs a, double* out29) {
  __shared__ double s_ne[kNE];
  __shared__ double s_nc[kLmWords];
  __shared__ double s_st[kLmWords];
  __shared__ double s_T[16];
  __shared__ int s_state;
  const Job& J = b.job[blockIdx.x];
  const MapDev& m = J.m;
  double* user_pose = J.pose;
  if (a.mode == 1) {
    if (threadIdx.x < kNE) out29[threadIdx.x] = fixed_total(acc_buf(m, a.acc_read) + threadIdx.x * kTermWords);
    return;
  }
  if (m.st->track_stop) {
    // stopped earlier: both scratch poses hold the last good pose
    if (a.mode == 0 && threadIdx.x < 16) user_pose[threadIdx.x] = pose_buf(m, user_pose, a.pose_read)[threadIdx.x];
    return;
  }
  if (a.mode == 2) {
    // the solve a tracking launch would run at its start, once per job
    if (a.adaptive) solve_step<true>(m, user_pose, a, J.stats, s_ne, s_T, &s_state, true, false, false, s_nc, s_st);
    else solve_step<false>(m, user_pose, a, J.stats, s_ne, s_T, &s_state, true, false, false, s_nc, s_st);
    return;
  }
  if (a.adaptive) solve_step<true>(m, user_pose, a, J.stats, s_ne, s_T, &s_state, true, false, true, s_nc, s_st);
  else solve_step<false>(m, user_pose, a, J.stats, s_ne, s_T, &s_state, true, false, false, s_nc, s_st);
}

__global__ void track_reset_kernel(Batch b) {
  const Job& J = b.job[blockIdx.x];
  for (int bi = 0; bi < 3; ++bi) {
    unsigned long long* acc = acc_buf(J.m, bi);
    for (int q = threadIdx.x; q < kUsedWords; q += blockDim.x) *used_word(acc, q) = 0ull;
  }
  if (threadIdx.x == 0) {
    J.m.st->track_stop = 0;
    J.m.st->track_counter = 0;
    rf_track_stats* stats = J.stats;
    if (stats) {
      stats->cost = 0.0;
      stats->count = 0.0;
      stats->iters = 0;
      stats->flags = 0;
      for (int l = 0; l < 8; ++l) stats->level_count[l] = 0.0;
    }
  }
}

// Tracking levels whose launches have more workgroups than this (all jobs
// together; two resident rounds of the chip) solve in a launch of their own,
// once per job, instead of redundantly at the start of every workgroup: with
// many workgroups the redundant solves and the reads of the accumulator
// copies they share cost more than the extra launch.  Both schedules run the
// same solve on the same totals, so the poses are identical.
constexpr int kSeparateSolveTiles = 3072;

static int track_tiles(const FrameDev& f, int level) {
  const int wl = (f.W + (1 << level) - 1) >> level;
  const int hl = (f.H + (1 << level) - 1) >> level;
  return ((wl + kTileW - 1) / kTileW) * ((hl + 15) >> 4);
}

static void track_dispatch(Batch& b, int df, int st, const TrackArgs& a, hipStream_t s) {
  int total = 0;
  for (int j = 0; j < b.n; ++j) {
    b.base[j] = total;
    total += track_tiles(b.job[j].f, a.level);
  }
  b.base[b.n] = total;
  const dim3 g(total), blk(kTrackBlock);
  auto run = [&](auto lm, auto slots) {
    constexpr bool L = decltype(lm)::value;
    constexpr int S = decltype(slots)::value;
    if (df == RF_DEPTH_U16) {
      if (st == RF_STORAGE_FP32) track_kernel<RF_DEPTH_U16, RF_STORAGE_FP32, L, S><<<g, blk, 0, s>>>(b, a);
      else track_kernel<RF_DEPTH_U16, RF_STORAGE_FP16_U8, L, S><<<g, blk, 0, s>>>(b, a);
    } else {
      if (st == RF_STORAGE_FP32) track_kernel<RF_DEPTH_F32, RF_STORAGE_FP32, L, S><<<g, blk, 0, s>>>(b, a);
      else track_kernel<RF_DEPTH_F32, RF_STORAGE_FP16_U8, L, S><<<g, blk, 0, s>>>(b, a);
    }
  };
  using Small = std::integral_constant<int, tile_refs(1) * 2>;
  using Large = std::integral_constant<int, kTileRefs>;
  static_assert(tile_refs(0) <= Small::value && tile_refs(1) <= Small::value, "level 0-1 pairs fit the small cache");
  const bool big = a.level >= 2;
  if (a.adaptive) {
    if (big) run(std::true_type{}, Large{});
    else run(std::true_type{}, Small{});
  } else {
    if (big) run(std::false_type{}, Large{});
    else run(std::false_type{}, Small{});
  }
}

void launch_track(Batch& b, int df, int st, const rf_track_params& tp, hipStream_t s) {
  track_reset_kernel<<<b.n, 256, 0, s>>>(b);
  int j = 0, prev_level = -1, prev_first = 0;
  for (int l = tp.levels - 1; l >= 0; --l) {
    int tiles = 0;
    for (int q = 0; q < b.n; ++q) tiles += track_tiles(b.job[q].f, l);
    const bool separate = tiles > kSeparateSolveTiles;
    for (int it = 0; it < tp.iters_per_level; ++it, ++j) {
      TrackArgs a{};
      a.level = l;
      a.w_c = tp.w_c;
      a.min_valid = tp.min_valid;
      a.lm_lambda = tp.lm_lambda;
      a.solve = j > 0;
      a.prev_level = prev_level;
      a.prev_first = prev_first;
      a.acc_read = j > 0 ? (j - 1) % 3 : -1;
      a.acc_write = j % 3;
      a.acc_clear = j > 0 ? (j + 1) % 3 : -1;
      a.pose_read = j > 0 ? (j - 1) % 2 : 2;
      a.pose_write = j % 2;
      a.mode = 0;
      a.adaptive = tp.adaptive;
      a.state_read = j > 0 ? (j - 1) % 2 : -1;
      a.state_write = j % 2;
      if (separate && a.solve) {
        // the solve once per job, then the evaluation at the pose it wrote
        TrackArgs c = a;
        c.mode = 2;
        track_finalize_kernel<<<b.n, 64, 0, s>>>(b, c, nullptr);
        a.solve = 0;
        a.pose_read = j % 2;
        a.pose_write = -1;
        a.state_write = -1;
      }
      track_dispatch(b, df, st, a, s);
      prev_level = l;
      prev_first = it == 0;
    }
  }
  if (j == 0) return;
  TrackArgs a{};
  a.level = -1;
  a.min_valid = tp.min_valid;
  a.lm_lambda = tp.lm_lambda;
  a.solve = 1;
  a.prev_level = prev_level;
  a.prev_first = prev_first;
  a.acc_read = (j - 1) % 3;
  a.acc_write = -1;
  a.acc_clear = -1;
  a.pose_read = (j - 1) % 2;
  a.pose_write = 2;
  a.adaptive = tp.adaptive;
  a.state_read = (j - 1) % 2;
  a.state_write = -1;
  track_finalize_kernel<<<b.n, 64, 0, s>>>(b, a, nullptr);
}

void launch_residual(Batch& b, int df, int st, float gamma, hipStream_t s) {
  int total = 0;
  for (int j = 0; j < b.n; ++j) {
    b.base[j] = total;
    total += track_tiles(b.job[j].f, 0);
  }
  b.base[b.n] = total;
  constexpr int S = tile_refs(1) * 2;  // the finest level's cache size, as in tracking
  static_assert(tile_refs(0) <= S, "level-0 pairs fit the cache");
  const dim3 g(total), blk(kTrackBlock);
  if (df == RF_DEPTH_U16) {
    if (st == RF_STORAGE_FP32) residual_kernel<RF_DEPTH_U16, RF_STORAGE_FP32, S><<<g, blk, 0, s>>>(b, gamma);
    else residual_kernel<RF_DEPTH_U16, RF_STORAGE_FP16_U8, S><<<g, blk, 0, s>>>(b, gamma);
  } else {
    if (st == RF_STORAGE_FP32) residual_kernel<RF_DEPTH_F32, RF_STORAGE_FP32, S><<<g, blk, 0, s>>>(b, gamma);
    else residual_kernel<RF_DEPTH_F32, RF_STORAGE_FP16_U8, S><<<g, blk, 0, s>>>(b, gamma);
  }
}

void launch_normal_equations(Batch& b, int df, int st, int level, float w_c, double* out29, hipStream_t s) {
  for (int j = 0; j < b.n; ++j) b.job[j].stats = nullptr;
  track_reset_kernel<<<b.n, 256, 0, s>>>(b);
  TrackArgs a{};
  a.level = level;
  a.w_c = w_c;
  a.solve = 0;
  a.acc_read = -1;
  a.acc_write = 0;
  a.acc_clear = -1;
  a.pose_read = 2;
  a.pose_write = 0;
  track_dispatch(b, df, st, a, s);
  TrackArgs c{};
  c.mode = 1;
  c.acc_read = 0;
  track_finalize_kernel<<<b.n, 64, 0, s>>>(b, c, out29);
}

}  // namespace rf
