// Host-side declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "refusion.h"
#include "rf_device.h"

namespace rf {

// Host view of one map: device pointers into the caller's arena plus the
// parameters every launch needs.
struct HostMap {
  rf_map_params p;
  void* arena;
  size_t bytes;
  MapDev dev;
  uint32_t frame_id;  // allocation epoch (frame stamps in the buckets)
};

void launch_allocate(const MapDev& m, const FrameDev& f, int depth_format, const double* pose,
                     const uint8_t* mask, uint32_t frame_id, hipStream_t s);
void launch_integrate(const MapDev& m, const FrameDev& f, int depth_format, int storage, const double* pose,
                      const uint8_t* mask, hipStream_t s);
void launch_track(const MapDev& m, const FrameDev& f, int depth_format, int storage,
                  const rf_track_params& tp, const uint8_t* mask, double* pose, rf_track_stats* stats,
                  hipStream_t s);
void launch_normal_equations(const MapDev& m, const FrameDev& f, int depth_format, int storage,
                             const uint8_t* mask, const double* pose, int level, float w_c, double* out29,
                             hipStream_t s);
void launch_mask(const MapDev& m, const FrameDev& f, int depth_format, int storage, const double* pose,
                 const rf_mask_params& mp, uint8_t* raw, uint8_t* eroded, uint8_t* filled, uint8_t* out,
                 float* residual, hipStream_t s);
void launch_map_init(const MapDev& m, uint32_t num_buckets, int storage, hipStream_t s);
void launch_surface(const MapDev& m, int storage, float* pts, uint32_t cap, uint32_t* count, hipStream_t s);
void launch_frame_blocks(const MapDev& m, int32_t* keys, uint32_t cap, uint32_t* count, hipStream_t s);
void launch_export(const MapDev& m, int storage, int32_t* keys, float* sdf, float* w, uint8_t* rgb,
                   uint32_t cap, uint32_t* count, hipStream_t s);
void launch_import(const MapDev& m, int storage, const int32_t* keys, const float* sdf, const float* w,
                   const uint8_t* rgb, uint32_t n, hipStream_t s);
int integrate_grid();

}  // namespace rf
