// Map maintenance kernels: initialisation, import/export (checkpoint), the
// frame block list, and zero-crossing surface extraction.
#include "rf_device.h"
#include "rf_internal.h"

namespace rf {

__global__ void init_buckets_kernel(Bucket* b, uint32_t n) {
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    Bucket e;
    e.key = kEmptyKey;
    e.slot = kInvalidSlot;
    e.pad = 0;
    b[i] = e;
  }
}

__global__ void zero_words_kernel(uint4* p, size_t n16) {
  const uint4 z = make_uint4(0, 0, 0, 0);
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
    p[i] = z;
}

__global__ void init_state_kernel(DevState* st) {
  if (threadIdx.x == 0) {
    st->n_blocks = 0;
    st->flags = 0;
    st->f_count = 0;
    st->track_counter = 0;
    st->track_stop = 0;
    st->dirty_count = 0;
    st->epoch = 0;
    st->n_band = 0;
    st->n_free = 0;
    st->cum_band = 0;
    st->cum_free = 0;
    st->cum_blocks = 0;
    st->cum_frames = 0;
    st->cum_whole = 0;
    st->n_keys = 0;
    st->w_count = 0;
    st->n_whole = 0;
  }
}

__global__ void init_refs_kernel(BlockRef* p, size_t n) {
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    p[i] = BlockRef{kEmptyKey, -1, 0u};
}

// Imported blocks end the allocation epoch, so no tracking cache keeps an
// absent-block entry across an import.
__global__ void advance_epoch_kernel(DevState* st) {
  if (threadIdx.x == 0) advance_epoch(st);
}

void launch_map_init(const MapDev& m, uint32_t num_buckets, int storage, hipStream_t s) {
  init_state_kernel<<<1, 64, 0, s>>>(m.st);
  init_refs_kernel<<<256, 256, 0, s>>>(m.tcache, (size_t)tile_refs_before(kCacheLevels) * m.tc_tiles);
  zero_words_kernel<<<16, 256, 0, s>>>(reinterpret_cast<uint4*>(m.tc_count), ((size_t)kCacheLevels * m.tc_tiles + 3) / 4);
  init_buckets_kernel<<<2048, 256, 0, s>>>(m.buckets, num_buckets);
  // no bucket touched; every listing leaves the map so
  zero_words_kernel<<<256, 256, 0, s>>>(reinterpret_cast<uint4*>(touched_map(m)), ((size_t)num_buckets + 15) / 16);
  // the flood-fill tile flags start at zero, and every mask computation
  // leaves them so
  zero_words_kernel<<<16, 256, 0, s>>>(reinterpret_cast<uint4*>(m.dirty), ((size_t)m.dirty_cap * 2 * 4 + 15) / 16);
  const size_t rec = (storage == RF_STORAGE_FP32) ? 8 : 4;
  zero_words_kernel<<<4096, 256, 0, s>>>(reinterpret_cast<uint4*>(m.sdfw), (size_t)m.max_blocks * 512 * rec / 16);
  zero_words_kernel<<<4096, 256, 0, s>>>(reinterpret_cast<uint4*>(m.rgb), (size_t)m.max_blocks * 512 * 4 / 16);
}

__device__ __forceinline__ uint32_t live_blocks(const MapDev& m) { return min(m.st->n_blocks, m.max_blocks); }

template <int STORAGE>
__global__ __launch_bounds__(256) void export_kernel(MapDev m, int32_t* keys, float* sdf, float* w, uint8_t* rgb,
                                                     uint32_t cap, uint32_t* count) {
  const uint32_t n = live_blocks(m);
  if (blockIdx.x == 0 && threadIdx.x == 0) *count = n;
  for (uint32_t b = blockIdx.x; b < n && b < cap; b += gridDim.x) {
    if (keys && threadIdx.x == 0) {
      int x, y, z;
      unpack_key(m.block_keys[b], x, y, z);
      keys[3 * b] = x;
      keys[3 * b + 1] = y;
      keys[3 * b + 2] = z;
    }
    for (int l = threadIdx.x; l < 512; l += blockDim.x) {
      const uint32_t i = b * 512u + l;
      float s, ww;
      VoxelStore<STORAGE>::load(m, i, s, ww);
      if (sdf) sdf[i] = s;
      if (w) w[i] = ww;
      if (rgb) {
        const uchar4 c = m.rgb[i];
        rgb[3 * (size_t)i] = c.x;
        rgb[3 * (size_t)i + 1] = c.y;
        rgb[3 * (size_t)i + 2] = c.z;
      }
    }
  }
}

template <int STORAGE>
__global__ __launch_bounds__(256) void import_kernel(MapDev m, const int32_t* keys, const float* sdf, const float* w,
                                                     const uint8_t* rgb, uint32_t n) {
  __shared__ int s_slot;
  for (uint32_t b = blockIdx.x; b < n; b += gridDim.x) {
    if (threadIdx.x == 0) {
      const int h = insert_block(m, keys[3 * b], keys[3 * b + 1], keys[3 * b + 2]);
      const uint32_t slot = (h >= 0) ? m.buckets[h].slot : kInvalidSlot;
      s_slot = (slot < m.max_blocks) ? (int)slot : -1;
    }
    __syncthreads();
    const int slot = s_slot;
    if (slot >= 0) {
      for (int l = threadIdx.x; l < 512; l += blockDim.x) {
        const size_t src = (size_t)b * 512 + l;
        const uint32_t dst = (uint32_t)slot * 512u + l;
        VoxelStore<STORAGE>::store(m, dst, sdf[src], w[src]);
        m.rgb[dst] = make_uchar4(rgb[3 * src], rgb[3 * src + 1], rgb[3 * src + 2], 0);
      }
    }
    __syncthreads();
  }
}

__global__ void frame_blocks_kernel(MapDev m, int32_t* keys, uint32_t cap, uint32_t* count) {
  const uint32_t n = min(m.st->f_count, m.flist_cap);
  if (blockIdx.x == 0 && threadIdx.x == 0) *count = n;
  for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n && i < cap; i += gridDim.x * blockDim.x) {
    int x, y, z;
    // compact free-space maps keep the whole-block test's outcome in bits 22-31
    unpack_key(m.buckets[m.flist[i] & (m.free_blocks ? 0x003FFFFFu : 0xFFFFFFFFu)].key, x, y, z);
    keys[3 * i] = x;
    keys[3 * i + 1] = y;
    keys[3 * i + 2] = z;
  }
}

__global__ void zero_u32_kernel(uint32_t* p) {
  if (threadIdx.x == 0) *p = 0;
}

template <int STORAGE>
__global__ __launch_bounds__(256) void surface_kernel(MapDev m, float* pts, uint32_t cap, uint32_t* count) {
  const uint32_t n = live_blocks(m);
  for (uint32_t b = blockIdx.x; b < n; b += gridDim.x) {
    int bx, by, bz;
    unpack_key(m.block_keys[b], bx, by, bz);
    for (int l = threadIdx.x; l < 512; l += blockDim.x) {
      const uint32_t i = b * 512u + l;
      float a, wa;
      VoxelStore<STORAGE>::load(m, i, a, wa);
      if (!(wa > 0.0f) || !(fabsf(a) < m.tau)) continue;
      const int lc[3] = {l & 7, (l >> 3) & 7, l >> 6};
      const int vi[3] = {8 * bx + lc[0], 8 * by + lc[1], 8 * bz + lc[2]};
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        uint32_t j;
        if (lc[ax] < 7) {
          j = i + (ax == 0 ? 1u : (ax == 1 ? 8u : 64u));
        } else {
          const int sl = find_slot(m, bx + (ax == 0), by + (ax == 1), bz + (ax == 2));
          if (sl < 0) continue;
          const int nl = (ax == 0 ? 0 : lc[0]) + 8 * (ax == 1 ? 0 : lc[1]) + 64 * (ax == 2 ? 0 : lc[2]);
          j = (uint32_t)sl * 512u + nl;
        }
        float c, wc;
        VoxelStore<STORAGE>::load(m, j, c, wc);
        if (!(wc > 0.0f) || !(fabsf(c) < m.tau)) continue;
        if ((a > 0.0f) == (c > 0.0f)) continue;
        const float tt = a / (a - c);
        const uint32_t k = atomicAdd(count, 1u);
        if (k < cap) {
          float* o = pts + 7 * (size_t)k;
          o[0] = (float)vi[0] * m.s;
          o[1] = (float)vi[1] * m.s;
          o[2] = (float)vi[2] * m.s;
          o[ax] = (float)vi[ax] * m.s + tt * m.s;
          const uchar4 col = m.rgb[i];
          o[3] = col.x;
          o[4] = col.y;
          o[5] = col.z;
          o[6] = (float)ax;
        }
      }
    }
  }
}

void launch_surface(const MapDev& m, int storage, float* pts, uint32_t cap, uint32_t* count, hipStream_t s) {
  zero_u32_kernel<<<1, 64, 0, s>>>(count);
  if (storage == RF_STORAGE_FP32) surface_kernel<RF_STORAGE_FP32><<<2048, 256, 0, s>>>(m, pts, cap, count);
  else surface_kernel<RF_STORAGE_FP16_U8><<<2048, 256, 0, s>>>(m, pts, cap, count);
}

// Free blocks of a compact free-space map: key and the weight their voxels
// read as, in no particular order (the buckets are scanned).
__global__ __launch_bounds__(256) void export_free_kernel(MapDev m, uint32_t num_buckets, int32_t* keys, float* w,
                                                          uint32_t cap, uint32_t* count) {
  for (uint32_t h = blockIdx.x * blockDim.x + threadIdx.x; h < num_buckets; h += gridDim.x * blockDim.x) {
    const Bucket b = m.buckets[h];
    if (b.key == kEmptyKey || !is_free_slot(b.slot)) continue;
    const uint32_t i = atomicAdd(count, 1u);
    if (i >= cap) continue;
    int x, y, z;
    unpack_key(b.key, x, y, z);
    keys[3 * i] = x;
    keys[3 * i + 1] = y;
    keys[3 * i + 2] = z;
    if (w) w[i] = (float)(b.slot & 0xFFu);
  }
}

void launch_export_free(const MapDev& m, uint32_t num_buckets, int32_t* keys, float* w, uint32_t cap, uint32_t* count,
                        hipStream_t s) {
  zero_u32_kernel<<<1, 64, 0, s>>>(count);
  export_free_kernel<<<2048, 256, 0, s>>>(m, num_buckets, keys, w, cap, count);
}

void launch_frame_blocks(const MapDev& m, int32_t* keys, uint32_t cap, uint32_t* count, hipStream_t s) {
  frame_blocks_kernel<<<256, 256, 0, s>>>(m, keys, cap, count);
}

void launch_export(const MapDev& m, int storage, int32_t* keys, float* sdf, float* w, uint8_t* rgb, uint32_t cap,
                   uint32_t* count, hipStream_t s) {
  if (storage == RF_STORAGE_FP32) export_kernel<RF_STORAGE_FP32><<<2048, 256, 0, s>>>(m, keys, sdf, w, rgb, cap, count);
  else export_kernel<RF_STORAGE_FP16_U8><<<2048, 256, 0, s>>>(m, keys, sdf, w, rgb, cap, count);
}

void launch_import(const MapDev& m, int storage, const int32_t* keys, const float* sdf, const float* w,
                   const uint8_t* rgb, uint32_t n, hipStream_t s) {
  if (n == 0) return;
  const int grid = (int)(n < 4096 ? n : 4096);
  advance_epoch_kernel<<<1, 64, 0, s>>>(m.st);
  if (storage == RF_STORAGE_FP32) import_kernel<RF_STORAGE_FP32><<<grid, 256, 0, s>>>(m, keys, sdf, w, rgb, n);
  else import_kernel<RF_STORAGE_FP16_U8><<<grid, 256, 0, s>>>(m, keys, sdf, w, rgb, n);
}

}  // namespace rf
