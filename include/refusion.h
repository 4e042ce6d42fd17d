/*
 * refusion.h -- C ABI of the MI355X (gfx950) implementation of the per-frame
 * hot path of ReFusion (Palazzolo, Behley, Lottes, Giguere, Stachniss,
 * "ReFusion: 3D Reconstruction in Dynamic Environments for RGB-D Cameras
 * Exploiting Residuals", IROS 2019).
 *
 * Per frame (the processing order of the paper's Fig. 2 and Section III):
 *   track_frame           (no mask)   initial registration, Sec. III-B
 *   compute_dynamic_mask               residual mask + flood fill, Sec. III-C
 *   track_frame           (with mask)  refined registration, Sec. III-C
 *   hashmap_allocate                   block allocation incl. carve rays, Sec. III-A/III-D
 *   integrate_frame                    running weighted average + carving, Sec. III-A/III-D
 * and, off the per-frame path, extract_surface (zero crossings), extract_mesh
 * (the model as a triangle mesh) and raycast_depth (virtual depth, Sec. III-E).
 *
 * Conventions shared by every call
 *  - All pointers named d_* and every buffer inside rf_frame are DEVICE
 *    pointers (HIP device memory of the current device); everything else is
 *    host memory.  The caller owns every buffer; the library keeps no pointer
 *    past the call except the map arena (until hashmap_destroy).
 *  - stream: a hipStream_t passed as void* (NULL = the null stream).  Calls
 *    only enqueue work; only map_status synchronises (the stream).
 *  - Poses are row-major 4x4 float64 matrices, camera -> world
 *    (y_world = R x_cam + t), stored in device memory (16 doubles).
 *  - Images are row-major, width fastest.  Depth: uint16 (x depth_scale
 *    metres, evaluated in FP32 as (float)raw * depth_scale) or float32 metres;
 *    0 (or > depth_max) marks an invalid pixel.  RGB: 3 interleaved uint8 per
 *    pixel.  Masks: uint8 per pixel, nonzero = dynamic (excluded).
 *  - Voxel v in Z^3 has its centre at v * voxel_size; block = floor(v / 8);
 *    a block holds 8^3 voxels with local index lx + 8 ly + 64 lz.
 *  - Return value: RF_OK, or a negative rf_status for argument, capacity or
 *    HIP errors detected on the host; then nothing was enqueued and
 *    rf_last_error() describes the problem.  Conditions found on the device
 *    (pool or hash full, degenerate tracking) are sticky bits in the map
 *    (map_status) and in rf_track_stats; they never abort a call.
 *  - A map must not be used from two streams at once; distinct maps are
 *    independent.
 */
#ifndef REFUSION_H
#define REFUSION_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t rf_status;
#define RF_OK 0
#define RF_EINVAL (-1)       /* bad argument or shape */
#define RF_ENOMEM (-2)       /* arena or caller buffer too small */
#define RF_EDEVICE (-3)      /* a HIP runtime call failed */
#define RF_EUNSUPPORTED (-4) /* valid request the library does not support */

/* sticky device-side condition bits (map_status, rf_track_stats.flags) */
#define RF_FLAG_POOL_FULL 0x1u        /* a block could not get a pool slot; its voxels are skipped */
#define RF_FLAG_HASH_FULL 0x2u        /* a key found no bucket within the probe limit */
#define RF_FLAG_TRACK_FEW_PIXELS 0x4u /* fewer than min_valid residuals: pass stopped, pose kept */
#define RF_FLAG_TRACK_SINGULAR 0x8u   /* Cholesky pivot <= 1e-12 trace(H): pass stopped, pose kept */
#define RF_FLAG_MASK_LIMIT 0x10u      /* flood-fill work limit reached (never expected) */
#define RF_FLAG_TRACK_RANGE 0x20u     /* a workgroup's normal-equation term was non-finite or |term| >= 2^34
                                         (beyond the fixed-point totals): pass stopped, pose kept */

#define RF_DEPTH_U16 0
#define RF_DEPTH_F32 1

#define RF_STORAGE_FP32 0    /* sdf float32 (metres), weight float32, colour RGB8 */
#define RF_STORAGE_FP16_U8 1 /* sdf float16 of sdf/truncation, weight uint8, colour RGB8 */

typedef struct {
  float fx, fy, cx, cy;   /* pinhole intrinsics (Eq. 1) */
  int32_t width, height;  /* pixels; width*height <= 2^26 and ceil(width/16)*ceil(height/16) <= 2^18 */
  const void* depth;      /* device, height*width of uint16 or float32 */
  int32_t depth_format;   /* RF_DEPTH_U16 | RF_DEPTH_F32 */
  float depth_scale;      /* metres per uint16 unit (e.g. 0.001); ignored for float32 */
  const uint8_t* rgb;     /* device, height*width*3 */
} rf_frame;

typedef struct {
  float voxel_size;       /* metres (edge of one voxel) */
  float truncation;       /* tau, metres: band half-width and the free-space value */
  float depth_max;        /* valid depth <= depth_max; also the carving clip plane */
  uint32_t num_buckets;   /* hash buckets, power of two */
  uint32_t max_blocks;    /* voxel-block pool capacity */
  uint32_t max_weight;    /* running-average weight cap, 1..255 */
  uint32_t carve_stride;  /* pixels (u,v) with u,v = 0 mod stride cast carve rays from the camera */
  int32_t storage;        /* RF_STORAGE_FP32 | RF_STORAGE_FP16_U8 */
  uint32_t max_pixels;    /* largest width*height passed to compute_dynamic_mask */
  int32_t free_blocks;    /* 1: compact free space (the free-space representation Sec. III-D leaves to
                             future work, as coarse free-block flags): a listed block whose image
                             rectangle holds only depths beyond it (+tau) is carved whole; a new block
                             keeps no voxels (a free block), its 512 voxels read as (sdf tau, weight =
                             frames that carved all of them, colour 0; unobserved while 0); it takes a
                             pool slot, its voxels starting from that value, the first time one of its
                             voxels gets a band update, and a frame that carves only some of its voxels
                             leaves it as it is.  Needs num_buckets <= 2^22.
                             0: every voxel carved by the per-voxel rule (Sec. III-D as written). */
} rf_map_params;

typedef struct {
  int32_t levels;          /* coarse-to-fine levels; level l uses every 2^l-th pixel (1..8) */
  int32_t iters_per_level; /* Gauss-Newton / LM iterations per level (fixed count) */
  float w_c;               /* weight of the photometric term, Eq. 4 */
  int32_t min_valid;       /* fewer residuals stop the pass (RF_FLAG_TRACK_FEW_PIXELS) */
  double lm_lambda;        /* damping: solves (H + lambda diag H) delta = -g; 0 = Gauss-Newton;
                              with adaptive = 1 the starting lambda */
  int32_t adaptive;        /* 0: every step is taken (Gauss-Newton, or fixed damping);
                              1: Levenberg-Marquardt (Sec. III-B): the first evaluation of a level is
                              accepted, a later candidate only with >= min_valid residuals and a mean
                              cost (cost/count) no larger than the accepted one (lambda /= 10), else
                              it is rejected (lambda = max(10 lambda, 1e-4)); steps start from the
                              accepted pose; the result is the last accepted pose */
} rf_track_params;

typedef struct {
  float gamma;  /* residual threshold t = gamma tau^2, Sec. III-C */
  float theta;  /* flood-fill depth ratio, Algorithm 1 */
} rf_mask_params;

typedef struct {
  double cost;            /* sum r_d^2 + w_c r_c^2 of the last evaluated iteration */
  double count;           /* residuals used in the last evaluated iteration */
  int32_t iters;          /* pose updates applied */
  uint32_t flags;         /* RF_FLAG_TRACK_* of this call */
  double level_count[8];  /* residuals used in the first iteration of each level */
} rf_track_stats;         /* written on the device */

typedef struct rf_map rf_map; /* opaque host handle */

/* ------------------------------------------------------------------------
 * Map (Sec. III-A): sparse TSDF of 8^3-voxel blocks in an open-addressed
 * spatial hash (linear probing, insert-only, as the paper never frees blocks).
 * ---------------------------------------------------------------------- */

/* Bytes of device memory a map with these parameters needs: the hash table,
 * the voxel pool and its colours, and scratch for tracking (accumulators and
 * a per-level, per-tile block cache of about 4 KiB per 256 pixels of
 * max_pixels), the dynamic mask and integration. */
rf_status hashmap_bytes(const rf_map_params* p, size_t* bytes);

/* Creates a map inside the caller's device arena (>= hashmap_bytes bytes,
 * 256-byte aligned) and enqueues its initialisation (empty hash, zeroed pool).
 * The arena stays owned by the caller and must outlive the map. */
rf_status hashmap_create(const rf_map_params* p, void* d_arena, size_t bytes, void* stream, rf_map** out);

/* Frees the host handle only. */
rf_status hashmap_destroy(rf_map* m);

/* Enqueues re-initialisation to the empty map (clears flags). */
rf_status hashmap_reset(rf_map* m, void* stream);

/* Block allocation for one frame (Sec. III-A, III-D).  For every valid pixel
 * with d_mask == 0 (d_mask may be NULL) a block-grid DDA visits the blocks of
 * the world segment of depths z in [max(D - tau, 0), D + tau] (pixels with
 * u, v = 0 mod carve_stride: z in [0, D + tau], so free space up to the
 * surface is covered); every visited block is inserted and recorded in the
 * frame's block list used by the next integrate_frame.  Pose d_pose: device.
 * A full pool or hash sets RF_FLAG_POOL_FULL / RF_FLAG_HASH_FULL and skips
 * that block. */
rf_status hashmap_allocate(rf_map* m, const rf_frame* f, const double* d_pose, const uint8_t* d_mask,
                           void* stream);

/* Integration (Sec. III-A, III-C, III-D) of the frame into every voxel of the
 * blocks listed by the preceding hashmap_allocate: the voxel projects to the
 * nearest pixel; eta = D - z; |eta| <= tau: sdf and colour are averaged with
 * d = eta; eta > tau and z <= depth_max: sdf is averaged toward tau (free
 * space); otherwise (eta < -tau, invalid or masked pixel, outside the image)
 * the voxel is untouched.  sdf <- (W sdf + d)/(W + 1), W <- min(W + 1,
 * max_weight); colour rounded half to even. */
rf_status integrate_frame(rf_map* m, const rf_frame* f, const double* d_pose, const uint8_t* d_mask,
                          void* stream);

/* Direct registration of the frame to the TSDF (Sec. III-B, Eqs. 1-4):
 * minimises sum S(T x)^2 + w_c (I_model(T x) - I(p))^2 over pixels with a
 * defined trilinear sample (all 8 corner voxels observed) and |S| < tau,
 * coarse to fine over `levels`, `iters_per_level` Gauss-Newton/LM steps each,
 * left update T <- exp(delta^) T.  d_pose_inout: device, initial pose in,
 * registered pose out.  d_mask: nullable, nonzero pixels are excluded (the
 * second registration).  d_stats: nullable device rf_track_stats.
 * Too few residuals or a singular system stop the call and keep the last
 * good pose (flags in d_stats). */
rf_status track_frame(rf_map* m, const rf_frame* f, const rf_track_params* tp, const uint8_t* d_mask,
                      double* d_pose_inout, rf_track_stats* d_stats, void* stream);

/* One evaluation of the normal equations at d_pose for pyramid level `level`
 * (Sec. III-B): d_out29 (device) receives H (21 upper-triangle terms,
 * row-major), g (6), cost and count as float64.  Diagnostic entry point. */
rf_status track_normal_equations(rf_map* m, const rf_frame* f, const uint8_t* d_mask, const double* d_pose,
                                 int32_t level, float w_c, double* d_out29, void* stream);

/* Dynamic mask (Sec. III-C): residual r = S(T x)^2 at pose d_pose for every
 * valid pixel with a defined sample; raw = r > gamma tau^2; 3x3 erosion;
 * depth-aware flood fill (Algorithm 1: a neighbour n of a member p joins when
 * |D(p) - D(n)| < theta D(p), 8-neighbourhood); 3x3 dilation.  Out-of-image
 * neighbours count as 0.  d_mask_out: device uint8 width*height.
 * d_residual_out: nullable device float32 width*height (-1 where undefined).
 * width*height must not exceed the map's max_pixels. */
rf_status compute_dynamic_mask(rf_map* m, const rf_frame* f, const double* d_pose, const rf_mask_params* mp,
                               uint8_t* d_mask_out, float* d_residual_out, void* stream);

/* compute_dynamic_mask for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * allocation): the same kernels and results, but the flood fill's scratch (a
 * per-pixel mask and two buffers of tile flags) lives in a static device
 * array of the library, 4 MiB per GPU, held until the process ends, instead
 * of the map arena.  The call allocates nothing.  Frames whose scratch
 * (width*height bytes rounded up to 256, plus 8 bytes per 32x32 tile) exceeds
 * 4 MiB -- about 4 million pixels -- are rejected with RF_ENOMEM before
 * anything is enqueued; the map's max_pixels does not limit this variant.
 * Every call on one GPU shares that GPU's array: calls that overlap on one
 * GPU (different streams, or host threads) race and must be serialised by
 * the caller.  Each call clears the tile flags it uses before the fill. */
rf_status compute_dynamic_mask_static(rf_map* m, const rf_frame* f, const double* d_pose, const rf_mask_params* mp,
                                      uint8_t* d_mask_out, float* d_residual_out, void* stream);

/* compute_dynamic_mask that also writes its intermediate masks (each nullable,
 * device uint8 width*height): raw threshold, eroded seeds M_R, flood fill M_D. */
rf_status compute_dynamic_mask_stages(rf_map* m, const rf_frame* f, const double* d_pose,
                                      const rf_mask_params* mp, uint8_t* d_raw, uint8_t* d_eroded,
                                      uint8_t* d_filled, uint8_t* d_mask_out, float* d_residual_out,
                                      void* stream);

/* Zero crossings of the TSDF on voxel edges (the surface the paper meshes):
 * for voxels v and v + e_axis both observed with |sdf| < tau and opposite
 * signs (sdf > 0 on one side only), the point v s + e_axis s sdf(v) /
 * (sdf(v) - sdf(v + e_axis)).  d_points: device float32 cap x 7 (x, y, z,
 * r, g, b of voxel v, axis); *d_count (device uint32) receives the total
 * number found (may exceed cap; only cap are written).  Order arbitrary. */
rf_status extract_surface(rf_map* m, float* d_points, uint32_t cap, uint32_t* d_count, void* stream);

/* Triangle mesh of the zero level set (the paper shows its models as meshes,
 * Sec. I and Fig. 1), by marching tetrahedra: a cube of 8 voxel centres is
 * meshed when all 8 voxels exist, are observed and hold |sdf| < tau; it is
 * cut into six tetrahedra along its diagonal (0, a, a|b, 7), inside means
 * sdf < 0, a crossing on an edge is interpolated linearly from the corner
 * with the fewer offset bits, and triangles face the positive side.  The
 * mesh is closed wherever the cubes are.  d_tris: device float32 cap x 9
 * (three vertices x, y, z in metres, counter-clockwise seen from the
 * positive side); *d_count (device uint32) receives the total triangle count,
 * which may exceed cap (then only the first cap are written: call again with
 * a larger buffer).  Enqueued on stream; uses the map's scratch, so calls on
 * one map must be ordered with its other calls.  Errors: RF_EINVAL for NULL
 * map/count or a NULL d_tris with cap > 0. */
rf_status extract_mesh(rf_map* m, float* d_tris, uint32_t cap, uint32_t* d_count, void* stream);

/* Virtual depth by ray casting the model (Sec. III-E, the second way to treat
 * invalid measurements: a model of the last n frames is cast from each
 * frame's registered pose and the frame's zero depths are replaced).  Along
 * pixel (u, v)'s ray the model is sampled (trilinear, defined where all 8
 * corner voxels are observed) at camera depths z_k = z_near + k tau/2,
 * z_k <= z_far; the virtual depth is the first crossing from a defined
 * sample S > 0 to the next defined sample S' <= 0, z + (tau/2) S / (S - S'),
 * or 0 without one.  f: the frame (intrinsics, size; its depth is read only
 * with only_invalid); d_pose: device float64 4x4 camera->world.  d_out:
 * device float32 width*height metres.  only_invalid = 1: pixels whose depth
 * is not zero keep it (in metres) and the zeros get the virtual depth, or
 * far_value where the ray meets no surface; only_invalid = 0: the virtual
 * depth of every pixel.  Errors: RF_EINVAL for NULL pointers, a bad frame,
 * z_near <= 0, z_far <= z_near, far_value < 0 or only_invalid not 0/1. */
rf_status raycast_depth(rf_map* m, const rf_frame* f, const double* d_pose, float z_near, float z_far,
                        float far_value, int32_t only_invalid, float* d_out, void* stream);

/* Sticky device flags (RF_FLAG_*) and allocated block count.  Synchronises
 * the stream. */
rf_status map_status(rf_map* m, void* stream, uint32_t* flags, uint32_t* n_blocks);

/* The blocks listed by the last hashmap_allocate (each once, in an order that
 * varies from run to run): d_keys (device int32, cap x 3 block coordinates);
 * *d_count (device uint32) = list length. */
rf_status hashmap_frame_blocks(rf_map* m, int32_t* d_keys, uint32_t cap, uint32_t* d_count, void* stream);

/* Export of every allocated block that holds voxels (checkpoint): d_keys
 * int32 cap x 3, d_sdf float32 cap x 512 (metres, decoded), d_weight float32
 * cap x 512, d_rgb uint8 cap x 512 x 3 (each device, nullable); *d_count
 * (device) = number of blocks (order arbitrary; only cap are written).  The
 * free blocks of a compact free-space map hold no voxels and are exported by
 * hashmap_export_free. */
rf_status hashmap_export(rf_map* m, int32_t* d_keys, float* d_sdf, float* d_weight, uint8_t* d_rgb,
                         uint32_t cap, uint32_t* d_count, void* stream);

/* Free blocks of a compact free-space map (rf_map_params.free_blocks = 1;
 * the free-space representation Sec. III-D leaves to future work): d_keys
 * (device int32, cap x 3 block coordinates), d_weight (device float32 cap,
 * nullable) = the weight all 512 voxels of the block read as (their sdf
 * reads as the truncation; 0 = not yet observed).  *d_count (device uint32)
 * = number of free blocks; order arbitrary, and when it exceeds cap, which
 * cap of them are written is unspecified.  A map without compact free space
 * has none. */
rf_status hashmap_export_free(rf_map* m, int32_t* d_keys, float* d_weight, uint32_t cap, uint32_t* d_count,
                              void* stream);

/* Import of n blocks in hashmap_export's layout (device arrays; keys must be
 * distinct).  Existing blocks with the same key are overwritten.  FP16
 * storage rounds sdf/tau to nearest even. */
rf_status hashmap_import(rf_map* m, const int32_t* d_keys, const float* d_sdf, const float* d_weight,
                         const uint8_t* d_rgb, uint32_t n, void* stream);

/* ------------------------------------------------------------------------
 * Batched forms (many sessions, one launch per stage).  Each job names its
 * own map, frame, device pose and buffers; a map may appear at most once per
 * call.  A job's results are identical (bit for bit) to the single-map call:
 * jobs share launches, never state.  Jobs are grouped internally by depth
 * format and storage and issued in launches of up to 8 jobs, in order.
 * ---------------------------------------------------------------------- */
typedef struct {
  rf_map* map;
  rf_frame frame;
  double* d_pose;           /* device 4x4 float64: in/out for tracking, read otherwise */
  const uint8_t* d_mask;    /* nullable input mask (registration pass 2, allocation, integration) */
  uint8_t* d_mask_out;      /* compute_dynamic_mask_batch output (width*height uint8) */
  rf_track_stats* d_stats;  /* nullable, track_frame_batch only */
} rf_job;

/* track_frame for every job (same rf_track_params for all). */
rf_status track_frame_batch(const rf_job* jobs, int32_t n, const rf_track_params* tp, void* stream);
/* compute_dynamic_mask for every job (writes d_mask_out). */
rf_status compute_dynamic_mask_batch(const rf_job* jobs, int32_t n, const rf_mask_params* mp, void* stream);
/* hashmap_allocate for every job (uses d_pose, d_mask). */
rf_status hashmap_allocate_batch(const rf_job* jobs, int32_t n, void* stream);
/* integrate_frame for every job (uses d_pose, d_mask); follows hashmap_allocate_batch. */
rf_status integrate_frame_batch(const rf_job* jobs, int32_t n, void* stream);

/* Thread-local description of the last error returned on this thread. */
const char* rf_last_error(void);

/* Library version string. */
const char* rf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* REFUSION_H */
