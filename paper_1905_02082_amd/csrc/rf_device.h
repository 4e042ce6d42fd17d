// Device-side data structures and helpers shared by the gfx950 kernels.
//
// Map layout in the caller's HBM arena (all sections 256-byte aligned):
//   DevState     counters and sticky flags
//   buckets      num_buckets x 16 B  {u64 packed block key, u32 pool slot, u32 pad}
//   touched      num_buckets x 1 B, buckets touched by the running allocation (right after them)
//   block_keys   max_blocks x 8 B    packed key of each pool slot
//   flist        num_buckets x 4 B   bucket indices of the blocks the last allocation touched
//   sdfw         max_blocks x 512 x  {f32 sdf, f32 weight} (FP32) | {f16 sdf/tau, u8 weight, pad} (FP16)
//   rgb          max_blocks x 512 x  uchar4 (RGB + pad)
//   partials     tracking: 3 buffers of 29 fixed-point accumulators (128 B apart) + 2 poses
//   mask scratch max_pixels bytes + two buffers of per-tile dirty flags for the flood fill
//   tile refs    tracking block cache: per level l < kCacheLevels, tc_tiles x tile_refs(l) x 16 B {key, slot, epoch},
//                then kCacheLevels x tc_tiles x 4 B pair counts
//   mesh scratch 2 x kMeshScratch x 4 B
//   cells        compact free space only: per 8x8 pixel cell of the frame, its smallest measured depth
//   wlist        compact free space only: num_buckets x 4 B, the integration's work list
//
// Hash: key = three 21-bit biased block coordinates; bucket = hash3 & mask,
// linear probing, insertion by 64-bit CAS on the key word (insert-only: keys
// never change once written, so a stale read can only show EMPTY, which the
// CAS then resolves).
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

#include "refusion.h"

namespace rf {

constexpr unsigned long long kEmptyKey = ~0ull;
constexpr uint32_t kInvalidSlot = 0xFFFFFFFFu;
// Compact free space: a bucket of a free block holds kFreeSlot | c instead of
// a pool slot, c = frames that carved it whole (capped at the weight cap).
constexpr uint32_t kFreeSlot = 0x80000000u;
__host__ __device__ __forceinline__ bool is_free_slot(uint32_t s) { return (s & 0xFFFFFF00u) == kFreeSlot; }
// Slot codes returned by resolve_slot: >= 0 pool slot, -1 absent (or no pool
// slot), <= -2 free block with count -2 - code.
__host__ __device__ __forceinline__ int free_code(uint32_t s) { return -2 - (int)(s & 0xFFu); }
constexpr int kKeyBias = 1 << 20;
constexpr float kMaxBlockCoord = 1.0e6f;   // |block coordinate| limit (key range 2^20)
constexpr float kMaxVoxelCoord = 8.0e6f;   // |voxel coordinate| limit (8 x 2^20 > 8e6)
#ifndef RF_TRACK_BLOCK
#define RF_TRACK_BLOCK 256
#endif
#ifndef RF_ACC_COPIES
#define RF_ACC_COPIES 8
#endif
constexpr int kTrackBlock = RF_TRACK_BLOCK;  // 256: 16x16 pixel tile; 512: 32x16
constexpr int kAccCopies = RF_ACC_COPIES;    // copies of the tracking accumulators
// 3 accumulator buffers + 2 poses + 2 Levenberg-Marquardt states (48 words each)
constexpr int kTrackScratchWords = 3 * kAccCopies * 29 * 16 + 32 + 2 * 48;
constexpr int kIntegGroups = 1536;  // integration workgroups per launch (all jobs together)
constexpr int kNE = 29;                    // 21 H + 6 g + cost + count
constexpr int kTile = 32;                  // flood-fill tile edge
constexpr int kCell = 8;                   // compact free space: depth-cell edge (pixels)

// Tracking block cache: for every pyramid level below kCacheLevels and every
// tracking tile, the (block key, pool slot) pairs its pixels looked up in the
// last launch at that level.  A pair of an existing block stays valid for
// good (blocks are never moved or removed; a reset or a new map clears the
// cache); an absent block is kept with slot -1 and the allocation epoch in
// which it was absent, and is valid only while that epoch lasts.
struct alignas(16) BlockRef {
  unsigned long long key;
  int slot;
  uint32_t epoch;
};
constexpr int kMeshScratch = 1024;  // workgroups of the mesh extraction
constexpr int kCacheLevels = 4;  // pyramid levels with a block cache
constexpr int kTileRefs = 512;   // largest pair capacity of a tile
// A 16x16 tile of level l covers 4^l times the area of a level-0 tile, so it
// touches more blocks: 64 pairs at level 0, 128 at level 1, 512 from level 2
// (a level-2 tile of 0.5 cm voxels touches ~110 blocks, up to ~230).
__host__ __device__ constexpr int tile_refs(int level) { return level >= 2 ? 512 : 64 << level; }
// First pair of level l's region, in units of tiles (region l holds
// tc_tiles x tile_refs(l) pairs).
__host__ __device__ constexpr int tile_refs_before(int level) {
  return level <= 0 ? 0 : tile_refs(level - 1) + tile_refs_before(level - 1);
}

struct alignas(16) Bucket {
  unsigned long long key;
  uint32_t slot;
  uint32_t pad;  // keeps a bucket one 16-byte load
};

struct DevState {
  uint32_t n_blocks;       // pool slots handed out (may exceed max_blocks when full)
  uint32_t flags;          // sticky RF_FLAG_*
  uint32_t f_count;        // entries in flist
  uint32_t track_counter;  // finished workgroups of the running tracking launch
  uint32_t track_stop;     // 1: the running registration pass stopped (degenerate)
  uint32_t dirty_count;    // flood fill: tiles marked since the last sweep
  uint32_t epoch;          // allocation epoch (frame stamps in the buckets), advanced on the device
  uint32_t n_keys;         // blocks inserted into the hash (with compact free space: free blocks too)
  unsigned long long n_band;  // voxels updated in the band by the last integration
  unsigned long long n_free;  // voxels carved by the last integration
  unsigned long long cum_band;    // since create/reset: band updates
  unsigned long long cum_free;    // since create/reset: free-space updates
  unsigned long long cum_blocks;  // since create/reset: listed blocks integrated
  unsigned long long cum_frames;  // since create/reset: integrations
  unsigned long long cum_whole;   // since create/reset: listed blocks carved whole (compact free space)
  uint32_t w_count;        // compact free space: entries in wlist
  uint32_t n_whole;        // compact free space: listed blocks carved whole by the running integration
};

// Starts a new allocation epoch (the tag of the tracking caches' entries for
// absent blocks, which an allocation may have inserted since); 0 is skipped
// on wrap.
__device__ __forceinline__ void advance_epoch(DevState* st) {
  const uint32_t e = st->epoch;
  st->epoch = (e == 0xFFFFFFFFu) ? 1u : e + 1u;
}

struct MapDev {
  Bucket* buckets;
  uint32_t bucket_mask;
  uint32_t max_probe;
  unsigned long long* block_keys;
  uint32_t* flist;
  uint32_t flist_cap;
  uint32_t max_blocks;
  void* sdfw;
  uchar4* rgb;
  DevState* st;
  double* partials;
  uint8_t* md;
  uint4* integ_counts;  // per integration workgroup: (band, free, 0, 0) updates of the last integration
  float* cells;         // compact free space: per 8x8 pixel cell of the frame being integrated, the
                        // smallest measured depth (0 if a pixel is masked or none is measured)
  uint32_t cells_cap;
  uint32_t free_blocks; // 1: compact free space
  uint32_t* wlist;      // compact free space: the frame-list entries left to the integration once the
                        // free blocks carved whole are counted (flist_cap entries)
  BlockRef* tcache;     // tracking block cache (per level: tc_tiles tiles of tile_refs(level) pairs)
  uint32_t* tc_count;   // valid pairs of each cached tile (kCacheLevels x tc_tiles)
  uint32_t* mesh_scratch;  // mesh extraction: triangles and offsets per workgroup (2 x kMeshScratch)
  uint32_t tc_tiles;    // tiles per level with a cache entry (later tiles look up the hash table only)
  uint32_t* dirty;
  uint32_t max_pixels;
  uint32_t dirty_cap;
  float s;        // voxel size
  float is;       // 1/s
  float iB;       // 1/(8 s)
  float tau;
  float inv_tau;
  float dmax;
  float max_weight;
  uint32_t carve_stride;
};

// Per bucket, 1 when the running allocation touched it: num_buckets bytes
// right after the buckets in the arena (the listing that follows the
// allocation clears what it lists).
__host__ __device__ __forceinline__ uint8_t* touched_map(const MapDev& m) {
  return reinterpret_cast<uint8_t*>(m.buckets + ((size_t)m.bucket_mask + 1));
}

struct FrameDev {
  const void* depth;
  const uint8_t* rgb;
  int W, H;
  float fx, fy, cx, cy;
  float ifx, ify;   // 1/fx, 1/fy in FP32
  float dscale;
};

// ---------------------------------------------------------------- keys
__device__ __forceinline__ unsigned long long pack_key(int x, int y, int z) {
  return ((unsigned long long)((uint32_t)(x + kKeyBias) & 0x1FFFFFu)) |
         (((unsigned long long)((uint32_t)(y + kKeyBias) & 0x1FFFFFu)) << 21) |
         (((unsigned long long)((uint32_t)(z + kKeyBias) & 0x1FFFFFu)) << 42);
}
__device__ __forceinline__ void unpack_key(unsigned long long k, int& x, int& y, int& z) {
  x = (int)(k & 0x1FFFFFull) - kKeyBias;
  y = (int)((k >> 21) & 0x1FFFFFull) - kKeyBias;
  z = (int)((k >> 42) & 0x1FFFFFull) - kKeyBias;
}
// Teschner et al. spatial hash of the block coordinate (uint32 wrap-around).
__device__ __forceinline__ uint32_t hash3(int x, int y, int z) {
  return ((uint32_t)x * 73856093u) ^ ((uint32_t)y * 19349669u) ^ ((uint32_t)z * 83492791u);
}

// Pool slot of block (x,y,z) or -1 (absent, a free block, or no slot because
// the pool was full).  Free blocks read as absent here: every voxel of one
// holds sdf = tau, which no zero-crossing test accepts.
__device__ __forceinline__ int find_slot(const MapDev& m, int x, int y, int z) {
  const unsigned long long key = pack_key(x, y, z);
  uint32_t h = hash3(x, y, z) & m.bucket_mask;
  for (uint32_t i = 0; i < m.max_probe; ++i) {
    const Bucket b = m.buckets[h];
    if (b.key == key) return (b.slot < m.max_blocks) ? (int)b.slot : -1;
    if (b.key == kEmptyKey) return -1;
    h = (h + 1) & m.bucket_mask;
  }
  return -1;
}

// Slot code of the key given the bucket b read at index h (its home bucket):
// continues the linear probe only when b holds another key.  >= 0 pool slot,
// -1 absent (or no pool slot), <= -2 free block (free_code).
__device__ __forceinline__ int resolve_slot(const MapDev& m, Bucket b, unsigned long long key, uint32_t h) {
  for (uint32_t i = 1;; ++i) {
    if (b.key == key) return (b.slot < m.max_blocks) ? (int)b.slot : (is_free_slot(b.slot) ? free_code(b.slot) : -1);
    if (b.key == kEmptyKey || i >= m.max_probe) return -1;
    h = (h + 1) & m.bucket_mask;
    b = m.buckets[h];
  }
}

// Inserts block (x,y,z) if absent; returns its bucket index or -1 (hash full).
// Probe from bucket h, whose key k the caller has already read, for block
// (x,y,z); insert it at the first empty bucket if absent.
__device__ __forceinline__ int find_or_insert_from(const MapDev& m, int x, int y, int z, uint32_t h,
                                                   unsigned long long k) {
  const unsigned long long key = pack_key(x, y, z);
  for (uint32_t i = 0; i < m.max_probe; ++i) {
    if (i > 0) k = m.buckets[h].key;
    if (k == key) return (int)h;
    if (k == kEmptyKey) {
      unsigned long long old = atomicCAS(&m.buckets[h].key, kEmptyKey, key);
      if (old == kEmptyKey) {
        atomicAdd(&m.st->n_keys, 1u);
        uint32_t slot;
        if (m.free_blocks) {
          slot = kFreeSlot;  // a free block: no voxels until one of them gets a band update
        } else {
          slot = atomicAdd(&m.st->n_blocks, 1u);
          if (slot < m.max_blocks) {
            m.block_keys[slot] = key;
          } else {
            slot = kInvalidSlot;
            atomicOr(&m.st->flags, (uint32_t)RF_FLAG_POOL_FULL);
          }
        }
        m.buckets[h].slot = slot;
        return (int)h;
      }
      if (old == key) return (int)h;
    }
    h = (h + 1) & m.bucket_mask;
  }
  atomicOr(&m.st->flags, (uint32_t)RF_FLAG_HASH_FULL);
  return -1;
}

// As find_or_insert_from, but a block this call inserts gets no pool slot
// and is not counted here (*claimed is set): the caller assigns slots and
// counts for a whole wavefront at once (one counter atomic instead of one
// per new block).  The probe starts i0 buckets past the home bucket `home`,
// whose key k the caller has already read.
__device__ __forceinline__ int find_or_claim_from(const MapDev& m, int x, int y, int z, uint32_t home, uint32_t i0,
                                                  unsigned long long k, bool* claimed) {
  const unsigned long long key = pack_key(x, y, z);
  *claimed = false;
  uint32_t h = (home + i0) & m.bucket_mask;
  // the keys past the known one are read two at a time (one round trip per
  // pair); a key read early may be one that another thread has since put
  // into an empty bucket, which the CAS below resolves as for any race
  unsigned long long kn = kEmptyKey;
  bool have_next = false;
  for (uint32_t i = i0; i < m.max_probe; ++i) {
    if (i > i0) {
      if (have_next) {
        k = kn;
        have_next = false;
      } else {
        k = m.buckets[h].key;
        if (i + 1 < m.max_probe) {
          kn = m.buckets[(h + 1) & m.bucket_mask].key;
          have_next = true;
        }
      }
    }
    if (k == key) return (int)h;
    if (k == kEmptyKey) {
      const unsigned long long old = atomicCAS(&m.buckets[h].key, kEmptyKey, key);
      if (old == kEmptyKey) {
        *claimed = true;
        return (int)h;
      }
      if (old == key) return (int)h;
    }
    h = (h + 1) & m.bucket_mask;
  }
  atomicOr(&m.st->flags, (uint32_t)RF_FLAG_HASH_FULL);
  return -1;
}

__device__ __forceinline__ int insert_block(const MapDev& m, int x, int y, int z) {
  const uint32_t h = hash3(x, y, z) & m.bucket_mask;
  return find_or_insert_from(m, x, y, z, h, m.buckets[h].key);
}

// ---------------------------------------------------------------- storage
template <int STORAGE>
struct VoxelStore;

template <>
struct VoxelStore<RF_STORAGE_FP32> {
  __device__ __forceinline__ static void load(const MapDev& m, uint32_t i, float& sdf, float& w) {
    const float2 v = reinterpret_cast<const float2*>(m.sdfw)[i];
    sdf = v.x;
    w = v.y;
  }
  __device__ __forceinline__ static void store(const MapDev& m, uint32_t i, float sdf, float w) {
    reinterpret_cast<float2*>(m.sdfw)[i] = make_float2(sdf, w);
  }
};

template <>
struct VoxelStore<RF_STORAGE_FP16_U8> {
  __device__ __forceinline__ static void load(const MapDev& m, uint32_t i, float& sdf, float& w) {
    const uint32_t v = reinterpret_cast<const uint32_t*>(m.sdfw)[i];
    sdf = __half2float(__ushort_as_half((unsigned short)(v & 0xFFFFu))) * m.tau;
    w = (float)((v >> 16) & 0xFFu);
  }
  __device__ __forceinline__ static void store(const MapDev& m, uint32_t i, float sdf, float w) {
    // The FP32 product is rounded first and then converted (two roundings, as
    // specified); the empty asm keeps the compiler from fusing the multiply
    // and the conversion into one mixed-precision FMA with a single rounding.
    float q = sdf * m.inv_tau;
    asm volatile("" : "+v"(q));
    const unsigned short h = __half_as_ushort(__float2half_rn(q));
    reinterpret_cast<uint32_t*>(m.sdfw)[i] = (uint32_t)h | ((uint32_t)w << 16);
  }
};

// ---------------------------------------------------------------- frame
template <int DF>
__device__ __forceinline__ float load_depth(const FrameDev& f, int idx) {
  if constexpr (DF == RF_DEPTH_U16) {
    return (float)reinterpret_cast<const uint16_t*>(f.depth)[idx] * f.dscale;
  } else {
    return reinterpret_cast<const float*>(f.depth)[idx];
  }
}
__device__ __forceinline__ bool depth_ok(float D, float dmax) { return D > 0.0f && D <= dmax; }

// Intensity in [0, 1] (Sec. III-B): ((0.2126 R + 0.7152 G) + 0.0722 B) / 255,
// correctly rounded.  The quotient is formed without a division: q = x RN(1/255)
// followed by one Newton correction q + (x - 255 q) RN(1/255) with both steps
// fused (Markstein); for every RGB8 colour this equals the correctly rounded
// x / 255 (checked exhaustively over all 2^24 colours on the CPU).
__device__ __forceinline__ float luminance(float r, float g, float b) {
  const float x = (0.2126f * r + 0.7152f * g) + 0.0722f * b;
  const float r255 = 1.0f / 255.0f;
  const float q = x * r255;
  return __builtin_fmaf(__builtin_fmaf(-q, 255.0f, x), r255, q);
}

// Correctly rounded a / b given y = RN(1/b): one fused Newton correction of
// the product a y (Markstein); with y the correctly rounded reciprocal the
// result equals the IEEE quotient for every a and b whose quotient is a
// normal number (checked exhaustively on the CPU for b = 1..256 and over
// random pairs for general b).
__device__ __forceinline__ float quotient_rn(float a, float b, float y) {
  const float q = a * y;
  return __builtin_fmaf(__builtin_fmaf(-q, b, a), y, q);
}

// Float copy of the FP64 pose: R row-major, t.
__device__ __forceinline__ void load_pose_f(const double* T, float R[9], float t[3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i) {
#pragma unroll
    for (int j = 0; j < 3; ++j) R[3 * i + j] = (float)T[4 * i + j];
    t[i] = (float)T[4 * i + 3];
  }
}

// y = R x + t evaluated as ((R0 x0 + R1 x1) + R2 x2) + t (no contraction).
__device__ __forceinline__ void xform(const float R[9], const float t[3], const float x[3], float y[3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i) y[i] = ((R[3 * i] * x[0] + R[3 * i + 1] * x[1]) + R[3 * i + 2] * x[2]) + t[i];
}

__device__ __forceinline__ float lerpf(float a, float b, float t) { return a + t * (b - a); }

// Trilinear interpolation of corner values c[k] (k = dx + 2 dy + 4 dz) at the
// fraction f; returns value and derivative with respect to the grid
// coordinate (x, then y, then z lerps).
__device__ __forceinline__ void trilinear(const float c[8], const float f[3], float& val, float dg[3],
                                          bool grad) {
  float cx00 = lerpf(c[0], c[1], f[0]);
  float cx01 = lerpf(c[2], c[3], f[0]);
  float cx10 = lerpf(c[4], c[5], f[0]);
  float cx11 = lerpf(c[6], c[7], f[0]);
  float cy0 = lerpf(cx00, cx01, f[1]);
  float cy1 = lerpf(cx10, cx11, f[1]);
  val = lerpf(cy0, cy1, f[2]);
  if (grad) {
    float dx00 = c[1] - c[0], dx01 = c[3] - c[2], dx10 = c[5] - c[4], dx11 = c[7] - c[6];
    float dxy0 = lerpf(dx00, dx01, f[1]);
    float dxy1 = lerpf(dx10, dx11, f[1]);
    dg[0] = lerpf(dxy0, dxy1, f[2]);
    float dy0 = cx01 - cx00, dy1 = cx11 - cx10;
    dg[1] = lerpf(dy0, dy1, f[2]);
    dg[2] = cy1 - cy0;
  }
}

// Pool slots of the distinct corner blocks of a trilinear lookup, from the
// hash table.  Corner k = dx + 2 dy + 4 dz lies in block (b0 + d) & cross; the
// distinct blocks are the corners k with k & ~cross == 0, and sl[k] of the
// others is copied from sl[k & cross].  The first probes are issued together
// (one round trip), and only collisions probe further.  Only the loaded key
// and slot stay live across the round trip; the key and home bucket are
// recomputed afterwards (cheaper than registers).  False if a block is absent.
struct HashSlots {
  __device__ __forceinline__ bool operator()(const MapDev& m, int bx0, int by0, int bz0, int cross, int sl[8]) const {
    unsigned long long bkey[8];
    uint32_t bslot[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if ((k & ~cross) != 0) continue;
      const int x = bx0 + (k & 1), y = by0 + ((k >> 1) & 1), z = bz0 + (k >> 2);
      const Bucket* p = m.buckets + (hash3(x, y, z) & m.bucket_mask);
      bkey[k] = p->key;
      bslot[k] = p->slot;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if ((k & ~cross) != 0) {
        sl[k] = sl[k & cross];
        continue;
      }
      const int x = bx0 + (k & 1), y = by0 + ((k >> 1) & 1), z = bz0 + (k >> 2);
      Bucket b0;
      b0.key = bkey[k];
      b0.slot = bslot[k];
      sl[k] = resolve_slot(m, b0, pack_key(x, y, z), hash3(x, y, z) & m.bucket_mask);
      if (sl[k] == -1) return false;
    }
    return true;
  }
};

// Voxel cell of world point y: lower corner voxel i0 and fractions fr;
// false outside the key range.
__device__ __forceinline__ bool voxel_cell(const MapDev& m, const float y[3], int i0[3], float fr[3]) {
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float g = y[a] * m.is;
    const float fl = floorf(g);
    if (!(fl > -kMaxVoxelCoord && fl < kMaxVoxelCoord)) return false;
    i0[a] = (int)fl;
    fr[a] = g - fl;
  }
  return true;
}

// The 8 corner records (and colours) of cell i0.  `slots` finds the slot
// codes of the corner blocks (HashSlots: the hash table; tracking adds a
// per-tile cache in front of it); false if a corner block is absent.  A
// corner in a free block (compact free space) reads (tau, count, colour 0),
// or unobserved while its count is 0.  All loads are issued before any is
// used, so they share one round trip.  With PIN the empty asm statements pin
// every loaded value here: without them the compiler sinks each load into the
// branch that first uses it, which turns the gathers back into a chain of
// round trips.  Without PIN the loads stay in flight for a later use (a
// speculative gather).
template <int STORAGE, bool WANT_COLOUR, bool PIN, class Slots>
__device__ __forceinline__ bool gather_corners(const MapDev& m, const int i0[3], const Slots& slots, float cs[8],
                                               float cw[8], uint32_t cc[8]) {
  const int bx0 = i0[0] >> 3, by0 = i0[1] >> 3, bz0 = i0[2] >> 3;
  const int cross = ((i0[0] & 7) == 7 ? 1 : 0) | ((i0[1] & 7) == 7 ? 2 : 0) | ((i0[2] & 7) == 7 ? 4 : 0);
  int sl[8];
  if (!slots(m, bx0, by0, bz0, cross, sl)) return false;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int dx = k & 1, dy = (k >> 1) & 1, dz = k >> 2;
    const uint32_t idx = (uint32_t)(sl[k] >= 0 ? sl[k] : 0) * 512u +
                         (uint32_t)(((i0[0] + dx) & 7) + 8 * ((i0[1] + dy) & 7) + 64 * ((i0[2] + dz) & 7));
    VoxelStore<STORAGE>::load(m, idx, cs[k], cw[k]);
    if (WANT_COLOUR) cc[k] = reinterpret_cast<const uint32_t*>(m.rgb)[idx];
  }
  if (PIN) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      asm volatile("" : "+v"(cs[k]), "+v"(cw[k]));
      if (WANT_COLOUR) asm volatile("" : "+v"(cc[k]));
    }
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    if (sl[k] >= 0) continue;  // free block
    const float c = (float)(-2 - sl[k]);
    cs[k] = c > 0.0f ? m.tau : 0.0f;
    cw[k] = c;
    if (WANT_COLOUR) cc[k] = 0u;
  }
  return true;
}

// Trilinear value (and gradient) of the corner records at fractions fr;
// defined only if all 8 corners are observed (weight > 0).  Gradients are
// with respect to world coordinates (d/dg * 1/s).
template <bool WANT_GRAD, bool WANT_COLOUR>
__device__ __forceinline__ bool interpolate(const MapDev& m, const float cs[8], const float cw[8],
                                            const uint32_t cc[8], const float fr[3], float& S, float gS[3],
                                            float& Iv, float gI[3]) {
  bool observed = true;
#pragma unroll
  for (int k = 0; k < 8; ++k) observed &= cw[k] > 0.0f;
  if (!observed) return false;
  float ci[8];
  if (WANT_COLOUR) {
#pragma unroll
    for (int k = 0; k < 8; ++k)
      ci[k] = luminance((float)(cc[k] & 0xFFu), (float)((cc[k] >> 8) & 0xFFu), (float)((cc[k] >> 16) & 0xFFu));
  }
  float dg[3];
  trilinear(cs, fr, S, dg, WANT_GRAD);
  if (WANT_GRAD) {
#pragma unroll
    for (int a = 0; a < 3; ++a) gS[a] = dg[a] * m.is;
  }
  if (WANT_COLOUR) {
    float di[3];
    trilinear(ci, fr, Iv, di, WANT_GRAD);
    if (WANT_GRAD) {
#pragma unroll
      for (int a = 0; a < 3; ++a) gI[a] = di[a] * m.is;
    }
  }
  return true;
}

// Trilinear sample of the TSDF (and, with WANT_COLOUR, of the model intensity)
// at world point y.  Defined only if all 8 corner voxels lie in allocated
// blocks and have weight > 0.
template <int STORAGE, bool WANT_GRAD, bool WANT_COLOUR, class Slots = HashSlots>
__device__ __forceinline__ bool sample_map(const MapDev& m, const float y[3], float& S, float gS[3],
                                           float& Iv, float gI[3], const Slots& slots = Slots()) {
  float fr[3];
  int i0[3];
  if (!voxel_cell(m, y, i0, fr)) return false;
  float cs[8], cw[8];
  uint32_t cc[8];
  if (!gather_corners<STORAGE, WANT_COLOUR, true>(m, i0, slots, cs, cw, cc)) return false;
  return interpolate<WANT_GRAD, WANT_COLOUR>(m, cs, cw, cc, fr, S, gS, Iv, gI);
}

}  // namespace rf
