// Seeded synthetic RGB-D renderer (test/benchmark input generator).
//
// Ray-casts analytic indoor scenes (room interior, oriented boxes, spheres,
// capsules) through a pinhole camera and writes depth, RGB8 and per-pixel
// "first hit is dynamic" labels.  Optionally adds the axial Kinect-style noise
// model sigma(z) = a + b (z - z0)^2, quantises to millimetres and drops a
// fraction of pixels to zero.  All randomness is counter-based (SplitMix64 of
// seed, frame, pixel, stream), so a frame does not depend on thread order.
//
// This module is only an input generator.  It contains none of the mapping
// method's arithmetic and is shared, as plain data, by the CPU oracle tests
// and the GPU tests/bench.
//
// Primitive record: 24 floats
//   [0] type: 0 room interior (axis-aligned box seen from inside),
//             1 box (yaw about world z), 2 sphere, 3 capsule
//   [1] label: 0 static, >0 id of the moving cluster
//   [2..4] centre, [5..7] half extents (box/room) or radius in [5]
//   [8],[9] cos(yaw), sin(yaw)
//   [10..12] albedo RGB in [0,1]
//   [13] texture spatial frequency (rad/m), [14..16] texture phases
//   [17..19] capsule half-axis (segment = centre -/+ axis)
#include <cmath>
#include <cstdint>
#include <cstring>
#include <algorithm>

namespace {

constexpr int kRec = 24;

inline uint64_t splitmix(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

inline double uniform01(uint64_t seed, int frame, int64_t pix, int stream) {
  uint64_t k = splitmix(splitmix(splitmix(seed) ^ (uint64_t)(uint32_t)frame) ^
                        (((uint64_t)pix << 3) | (uint64_t)stream));
  return (double)(k >> 11) * (1.0 / 9007199254740992.0);
}

struct Hit {
  double t = INFINITY;
  const float* prim = nullptr;
};

inline double dot3(const double* a, const double* b) { return a[0]*b[0] + a[1]*b[1] + a[2]*b[2]; }

// Exit distance of a ray that starts inside an axis-aligned box.
double room_exit(const float* p, const double* o, const double* d) {
  double t = INFINITY;
  for (int i = 0; i < 3; ++i) {
    double lo = p[2+i] - p[5+i], hi = p[2+i] + p[5+i];
    if (d[i] > 0) t = std::min(t, (hi - o[i]) / d[i]);
    else if (d[i] < 0) t = std::min(t, (lo - o[i]) / d[i]);
  }
  return t;
}

double box_enter(const float* p, const double* o, const double* d) {
  double c = p[8], s = p[9];
  double oc[3] = {o[0]-p[2], o[1]-p[3], o[2]-p[4]};
  // rotate by -yaw into the box frame
  double ol[3] = { c*oc[0] + s*oc[1], -s*oc[0] + c*oc[1], oc[2] };
  double dl[3] = { c*d[0] + s*d[1],  -s*d[0] + c*d[1],  d[2] };
  double tmin = -INFINITY, tmax = INFINITY;
  for (int i = 0; i < 3; ++i) {
    double h = p[5+i];
    if (dl[i] == 0) {
      if (ol[i] < -h || ol[i] > h) return INFINITY;
      continue;
    }
    double t1 = (-h - ol[i]) / dl[i], t2 = (h - ol[i]) / dl[i];
    if (t1 > t2) std::swap(t1, t2);
    tmin = std::max(tmin, t1);
    tmax = std::min(tmax, t2);
  }
  if (tmax < tmin || tmin <= 1e-9) return INFINITY;
  return tmin;
}

double sphere_enter(const double* c, double r, const double* o, const double* d) {
  double oc[3] = {o[0]-c[0], o[1]-c[1], o[2]-c[2]};
  double a = dot3(d, d), b = dot3(d, oc), cc = dot3(oc, oc) - r*r;
  double disc = b*b - a*cc;
  if (disc < 0) return INFINITY;
  double t = (-b - std::sqrt(disc)) / a;
  return t > 1e-9 ? t : INFINITY;
}

double capsule_enter(const float* p, const double* o, const double* d) {
  double p0[3], p1[3];
  for (int i = 0; i < 3; ++i) { p0[i] = p[2+i] - p[17+i]; p1[i] = p[2+i] + p[17+i]; }
  double r = p[5];
  double ba[3] = {p1[0]-p0[0], p1[1]-p0[1], p1[2]-p0[2]};
  double oa[3] = {o[0]-p0[0], o[1]-p0[1], o[2]-p0[2]};
  double baba = dot3(ba, ba), bard = dot3(ba, d), baoa = dot3(ba, oa);
  double rdoa = dot3(d, oa), oaoa = dot3(oa, oa), dd = dot3(d, d);
  double a = baba*dd - bard*bard;
  double b = baba*rdoa - baoa*bard;
  double c = baba*oaoa - baoa*baoa - r*r*baba;
  double best = INFINITY;
  if (a > 1e-12) {
    double h = b*b - a*c;
    if (h >= 0) {
      double t = (-b - std::sqrt(h)) / a;
      double y = baoa + t*bard;
      if (t > 1e-9 && y > 0 && y < baba) best = t;
    }
  }
  best = std::min(best, sphere_enter(p0, r, o, d));
  best = std::min(best, sphere_enter(p1, r, o, d));
  return best;
}

void shade(const float* p, const double* x, uint8_t* rgb) {
  double f = p[13];
  double l[3] = {x[0]-p[2], x[1]-p[3], x[2]-p[4]};
  double s = (std::sin(f*l[0] + p[14]) + std::sin(f*l[1] + p[15]) + std::sin(f*l[2] + p[16])) / 3.0;
  double k = 0.6 + 0.4*s;
  for (int i = 0; i < 3; ++i) {
    double v = std::round(255.0 * std::min(1.0, std::max(0.0, p[10+i]*k)));
    rgb[i] = (uint8_t)v;
  }
}

}  // namespace

extern "C" {

// Renders frames [0, n_frames) of a sequence.  prims: n_frames x n_prims x 24
// floats (each frame carries its own primitive placement so moving clusters can
// be posed per frame); poses: n_frames x 16 doubles, row-major camera->world.
// noise_a/noise_b/noise_z0: sigma(z) = a + b (z - z0)^2 (a = b = 0: no noise).
// depth_f32 (n x H x W, metres, noise-free) and depth_u16 (millimetres, noisy,
// quantised, clipped to [min_mm, max_mm], with dropout) may each be null.
// Returns 0 on success.
int synth_render(const float* prims, int n_prims, const double* poses, int n_frames,
                 int W, int H, double fx, double fy, double cx, double cy,
                 uint64_t seed, int frame0, double noise_a, double noise_b, double noise_z0,
                 double dropout, int min_mm, int max_mm,
                 float* depth_f32, uint16_t* depth_u16, uint8_t* rgb, uint8_t* labels) {
  if (W <= 0 || H <= 0 || n_frames < 0 || n_prims <= 0) return -1;
#pragma omp parallel for collapse(2) schedule(dynamic, 4)
  for (int f = 0; f < n_frames; ++f) {
    for (int v = 0; v < H; ++v) {
      const double* T = poses + 16*(int64_t)f;
      const float* P = prims + (int64_t)f*n_prims*kRec;
      const int frame = frame0 + f;
      for (int u = 0; u < W; ++u) {
        int64_t pix = (int64_t)v*W + u;
        int64_t o_idx = (int64_t)f*W*H + pix;
        double dc[3] = {(u - cx)/fx, (v - cy)/fy, 1.0};
        double o[3] = {T[3], T[7], T[11]};
        double d[3];
        for (int i = 0; i < 3; ++i) d[i] = T[4*i]*dc[0] + T[4*i+1]*dc[1] + T[4*i+2]*dc[2];
        Hit hit;
        for (int k = 0; k < n_prims; ++k) {
          const float* p = P + k*kRec;
          double t = INFINITY;
          switch ((int)p[0]) {
            case 0: t = room_exit(p, o, d); break;
            case 1: t = box_enter(p, o, d); break;
            case 2: { double c[3] = {p[2], p[3], p[4]}; t = sphere_enter(c, p[5], o, d); } break;
            case 3: t = capsule_enter(p, o, d); break;
            default: break;
          }
          if (t < hit.t) { hit.t = t; hit.prim = p; }
        }
        uint8_t* px = rgb + 3*o_idx;
        if (!hit.prim || !std::isfinite(hit.t)) {
          px[0] = px[1] = px[2] = 0;
          if (depth_f32) depth_f32[o_idx] = 0.f;
          if (depth_u16) depth_u16[o_idx] = 0;
          if (labels) labels[o_idx] = 0;
          continue;
        }
        double x[3] = {o[0] + hit.t*d[0], o[1] + hit.t*d[1], o[2] + hit.t*d[2]};
        shade(hit.prim, x, px);
        if (labels) labels[o_idx] = (uint8_t)std::min(255.f, hit.prim[1]);
        double z = hit.t;  // the camera-frame z of the hit, since dc.z == 1
        if (depth_f32) depth_f32[o_idx] = (float)z;
        if (depth_u16) {
          double zn = z;
          if (noise_a > 0 || noise_b > 0) {
            double sig = noise_a + noise_b*(z - noise_z0)*(z - noise_z0);
            double u1 = std::max(uniform01(seed, frame, pix, 0), 1e-300);
            double u2 = uniform01(seed, frame, pix, 1);
            zn = z + sig*std::sqrt(-2.0*std::log(u1))*std::cos(6.283185307179586*u2);
          }
          long mm = std::lround(zn*1000.0);
          if (mm < min_mm || mm > max_mm) mm = 0;
          if (dropout > 0 && uniform01(seed, frame, pix, 2) < dropout) mm = 0;
          depth_u16[o_idx] = (uint16_t)mm;
        }
      }
    }
  }
  return 0;
}

}  // extern "C"
