// Host-side declarations shared by the library's translation units, and the
// job batch every per-frame kernel consumes.
//
// Every per-frame kernel works on a batch of up to kMaxBatch jobs passed by
// value as a kernel argument (a job = one map + one frame + its pose, mask
// and outputs).  The grid is the concatenation of the jobs' grids: base[j] is
// the first workgroup of job j.  A single-map call is a batch of one, so the
// multi-session path and the single-session path run the same kernels; a
// job's result never depends on the other jobs in its batch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "refusion.h"
#include "rf_device.h"

namespace rf {

constexpr int kMaxBatch = 8;

struct Job {
  MapDev m;
  FrameDev f;
  const uint8_t* mask;      // input mask (nullable)
  double* pose;             // device pose (in/out for tracking)
  rf_track_stats* stats;    // nullable
  uint8_t* mask_out;        // dynamic mask outputs
  uint8_t* raw;
  uint8_t* eroded;
  uint8_t* filled;
  float* residual;
  int tiles_x, tiles_y;     // flood-fill tile grid
  int carve_groups;         // allocation: workgroups of carve rays (before the band rays')
  int carve_w, carve_h;     // allocation: carve-grid size
  int cells_w, cells_h;     // integration of a compact free-space map: 8x8 depth cells of the frame
};

struct Batch {
  int n;
  int base[kMaxBatch + 1];
  Job job[kMaxBatch];
};

static_assert(sizeof(Batch) <= 3072, "job batch must stay well inside the kernel-argument limit");

// Job of workgroup g (uniform per workgroup).
__device__ __forceinline__ int batch_job(const Batch& b, int g) {
  int j = 0;
  while (j + 1 < b.n && g >= b.base[j + 1]) ++j;
  return j;
}

// Host view of one map: device pointers into the caller's arena plus the
// parameters every launch needs.
struct HostMap {
  rf_map_params p;
  void* arena;
  size_t bytes;
  MapDev dev;
};

// Launchers: b holds 1..kMaxBatch jobs sharing depth format and storage.
void launch_allocate(Batch& b, int depth_format, hipStream_t s);
void launch_integrate(Batch& b, int depth_format, int storage, hipStream_t s);
void launch_track(Batch& b, int depth_format, int storage, const rf_track_params& tp, hipStream_t s);
void launch_normal_equations(Batch& b, int depth_format, int storage, int level, float w_c, double* out29,
                             hipStream_t s);
void launch_mask(Batch& b, int depth_format, int storage, const rf_mask_params& mp, hipStream_t s);
// residual and raw decision of the mask (its first stage), through the tracking tile cache
void launch_residual(Batch& b, int depth_format, int storage, float gamma, hipStream_t s);

void launch_map_init(const MapDev& m, uint32_t num_buckets, int storage, hipStream_t s);
void launch_surface(const MapDev& m, int storage, float* pts, uint32_t cap, uint32_t* count, hipStream_t s);
void launch_mesh(const MapDev& m, int storage, float* tris, uint32_t cap, uint32_t* count, hipStream_t s);
void launch_raycast(const MapDev& m, const FrameDev& f, int depth_format, int storage, const double* pose,
                    float z_near, float z_far, float far_value, int only_invalid, float* out, hipStream_t s);
void launch_frame_blocks(const MapDev& m, int32_t* keys, uint32_t cap, uint32_t* count, hipStream_t s);
void launch_export_free(const MapDev& m, uint32_t num_buckets, int32_t* keys, float* w, uint32_t cap, uint32_t* count,
                        hipStream_t s);
void launch_export(const MapDev& m, int storage, int32_t* keys, float* sdf, float* w, uint8_t* rgb,
                   uint32_t cap, uint32_t* count, hipStream_t s);
void launch_import(const MapDev& m, int storage, const int32_t* keys, const float* sdf, const float* w,
                   const uint8_t* rgb, uint32_t n, hipStream_t s);

}  // namespace rf
