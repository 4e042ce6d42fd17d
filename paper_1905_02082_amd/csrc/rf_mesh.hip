// Triangle mesh of the model's zero level set (the paper shows its models as
// meshes, Sec. I and Fig. 1) by marching tetrahedra, for gfx950.
//
// A cube of 8 voxel centres (lower corner v, corner k = dx + 2 dy + 4 dz at
// v + (dx, dy, dz)) is meshed when all 8 voxels exist, are observed (w > 0)
// and hold |sdf| < tau.  It is cut into the six tetrahedra (0, a, a|b, 7)
// along its diagonal, one per order of the axis bits; neighbouring cubes cut
// their shared faces alike, so the mesh is closed wherever the cubes are.
// Inside means sdf < 0.  One vertex alone on its side gives a triangle (the
// crossings of its three edges), two and two a quad (two triangles).  The
// crossing on edge (a, b), a the corner whose bits are a subset of b's, is
// P_a + t (P_b - P_a) with t = f_a / (f_a - f_b), so every tetrahedron and
// cube that shares a grid edge computes the same point.  Triangles face the
// positive (observed) side: a triangle whose normal has a negative dot
// product with n_in * sum(outside corners) - n_out * sum(inside corners) is
// reversed.
//
// Three launches, so that the output is compact without a contended
// counter: a count pass (triangles per workgroup), a one-workgroup scan, and
// a write pass in which every workgroup walks its blocks in the same order
// and places each thread's triangles by a prefix sum over the workgroup.
// Given the pool order of the blocks the output order is deterministic.
#include "rf_device.h"
#include "rf_internal.h"

namespace rf {

constexpr int kMeshThreads = 512;  // one thread per voxel cube of a block

// Corner j of tetrahedron t: the chain 0, a, a|b, 7 with first axis bit
// a = 1 << (t / 2) and second b the lower (t even) or higher (t odd) of the
// other two bits: (0,1,3,7) (0,1,5,7) (0,2,3,7) (0,2,6,7) (0,4,5,7) (0,4,6,7).
__host__ __device__ constexpr int tet_corner(int t, int j) {
  return j == 0 ? 0
                : (j == 3 ? 7
                          : ((1 << (t >> 1)) |
                             (j == 1 ? 0
                                     : ((t & 1) ? ((7 & ~(1 << (t >> 1))) & ~((7 & ~(1 << (t >> 1))) & -(7 & ~(1 << (t >> 1)))))
                                                : ((7 & ~(1 << (t >> 1))) & -(7 & ~(1 << (t >> 1))))))));
}
static_assert(tet_corner(0, 2) == 3 && tet_corner(1, 2) == 5 && tet_corner(2, 2) == 3 && tet_corner(3, 2) == 6 &&
                  tet_corner(4, 2) == 5 && tet_corner(5, 2) == 6 && tet_corner(5, 1) == 4,
              "tetrahedra of the cube");

// f[k] for a corner index known only at run time (a select chain, so the
// corner values stay in registers).
__device__ __forceinline__ float pick(const float f[8], int k) {
  float r = f[0];
#pragma unroll
  for (int i = 1; i < 8; ++i) r = (k == i) ? f[i] : r;
  return r;
}

// SDF of the 8 corners of the cube with lower corner at local voxel l of the
// block whose neighbour slots (block offset dx + 2 dy + 4 dz) are nb; false
// unless every corner exists, is observed and holds |sdf| < tau.
template <int STORAGE>
__device__ __forceinline__ bool cube_corners(const MapDev& m, const int* nb, int l, float f[8]) {
  const int lx = l & 7, ly = (l >> 3) & 7, lz = l >> 6;
  float w[8];
  bool ok = true;
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int cx = lx + (k & 1), cy = ly + ((k >> 1) & 1), cz = lz + (k >> 2);
    const int sl = nb[(cx >> 3) | ((cy >> 3) << 1) | ((cz >> 3) << 2)];
    ok &= sl >= 0;
    const uint32_t idx = (uint32_t)(sl >= 0 ? sl : 0) * 512u + (uint32_t)((cx & 7) + 8 * (cy & 7) + 64 * (cz & 7));
    VoxelStore<STORAGE>::load(m, idx, f[k], w[k]);
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) ok &= w[k] > 0.0f && fabsf(f[k]) < m.tau;
  return ok;
}

__device__ __forceinline__ int tet_triangles(const float f[8], int t) {
  int ni = 0;
#pragma unroll
  for (int j = 0; j < 4; ++j) ni += f[tet_corner(t, j)] < 0.0f ? 1 : 0;
  return (ni == 1 || ni == 3) ? 1 : (ni == 2 ? 2 : 0);
}

__device__ __forceinline__ int cube_count(const float f[8]) {
  int n = 0;
#pragma unroll
  for (int t = 0; t < 6; ++t) n += tet_triangles(f, t);
  return n;
}

// Corner k's position, component a (voxel centres at v s).
__device__ __forceinline__ float corner_pos(const int v[3], int k, int a, float s) {
  return (float)(v[a] + ((k >> a) & 1)) * s;
}

struct MeshOut {
  float* tris;
  uint32_t cap;
  uint32_t next;  // index of the next triangle this thread writes
  __device__ __forceinline__ void emit(const float* q0, const float* q1, const float* q2) {
    if (next < cap) {
      float* o = tris + 9 * (size_t)next;
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        o[a] = q0[a];
        o[3 + a] = q1[a];
        o[6 + a] = q2[a];
      }
    }
    ++next;
  }
};

__device__ __forceinline__ void cube_write(const float f[8], const int v[3], float s, MeshOut& out) {
#pragma unroll
  for (int t = 0; t < 6; ++t) {
    // inside and outside corners in tetrahedron order, 4 bits each
    uint32_t insp = 0u, outp = 0u;
    int ni = 0, no = 0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int k = tet_corner(t, j);
      if (f[k] < 0.0f) {
        insp |= (uint32_t)k << (4 * ni);
        ++ni;
      } else {
        outp |= (uint32_t)k << (4 * no);
        ++no;
      }
    }
    if (ni == 0 || no == 0) continue;
    auto in_at = [&](int j) { return (int)((insp >> (4 * j)) & 15u); };
    auto out_at = [&](int j) { return (int)((outp >> (4 * j)) & 15u); };
    // crossing point of the edge between corners i and o (from the subset corner)
    auto cross = [&](int i, int o, float* q) {
      const int lo = (i & o) == i ? i : o, hi = lo == i ? o : i;
      const float fl = pick(f, lo), fh = pick(f, hi);
      const float tt = fl / (fl - fh);
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const float pl = corner_pos(v, lo, a, s), ph = corner_pos(v, hi, a, s);
        q[a] = pl + tt * (ph - pl);
      }
    };
    float ref[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      float so = 0.0f, si = 0.0f;
#pragma unroll
      for (int j = 0; j < 3; ++j)
        if (j < no) so += corner_pos(v, out_at(j), a, s);
#pragma unroll
      for (int j = 0; j < 3; ++j)
        if (j < ni) si += corner_pos(v, in_at(j), a, s);
      ref[a] = (float)ni * so - (float)no * si;
    }
    auto facing = [&](const float* q0, const float* q1, const float* q2) {
      const float e1[3] = {q1[0] - q0[0], q1[1] - q0[1], q1[2] - q0[2]};
      const float e2[3] = {q2[0] - q0[0], q2[1] - q0[1], q2[2] - q0[2]};
      const float nx = e1[1] * e2[2] - e1[2] * e2[1], ny = e1[2] * e2[0] - e1[0] * e2[2],
                  nz = e1[0] * e2[1] - e1[1] * e2[0];
      return (nx * ref[0] + ny * ref[1]) + nz * ref[2] >= 0.0f;
    };
    if (ni == 1 || no == 1) {
      const int lone = ni == 1 ? in_at(0) : out_at(0);
      float q[3][3];
#pragma unroll
      for (int j = 0; j < 3; ++j) cross(lone, ni == 1 ? out_at(j) : in_at(j), q[j]);
      if (facing(q[0], q[1], q[2])) out.emit(q[0], q[1], q[2]);
      else out.emit(q[0], q[2], q[1]);
    } else {
      float q[4][3];
      cross(in_at(0), out_at(0), q[0]);
      cross(in_at(0), out_at(1), q[1]);
      cross(in_at(1), out_at(1), q[2]);
      cross(in_at(1), out_at(0), q[3]);
      if (facing(q[0], q[1], q[2])) {
        out.emit(q[0], q[1], q[2]);
        out.emit(q[0], q[2], q[3]);
      } else {
        out.emit(q[0], q[2], q[1]);
        out.emit(q[0], q[3], q[2]);
      }
    }
  }
}

// Slots of block b and of its 7 upper neighbours (threads 0..7), in LDS.
__device__ __forceinline__ void neighbour_slots(const MapDev& m, uint32_t b, int bx, int by, int bz, int* s_nb) {
  const int t = threadIdx.x;
  if (t < 8) s_nb[t] = t == 0 ? (int)b : find_slot(m, bx + (t & 1), by + ((t >> 1) & 1), bz + (t >> 2));
}

// The same for block b if b < n (the walks look one block ahead: the next
// block's hash probes run while the current block's corner records load).
__device__ __forceinline__ void prefetch_slots(const MapDev& m, uint32_t b, uint32_t n, int* s_nb) {
  if (b < n && threadIdx.x < 8) {
    int bx, by, bz;
    unpack_key(m.block_keys[b], bx, by, bz);
    neighbour_slots(m, b, bx, by, bz, s_nb);
  }
}

// Pass 1: triangles per workgroup -> scratch[g].
template <int STORAGE>
__global__ __launch_bounds__(kMeshThreads) void mesh_count_kernel(MapDev m, uint32_t* scratch) {
  __shared__ int s_nb[2][8];
  __shared__ uint32_t s_sum;
  if (threadIdx.x == 0) s_sum = 0u;
  const uint32_t n = min(m.st->n_blocks, m.max_blocks);
  prefetch_slots(m, blockIdx.x, n, s_nb[0]);
  uint32_t mine = 0;
  int cur = 0;
  for (uint32_t b = blockIdx.x; b < n; b += gridDim.x, cur ^= 1) {
    // this block's slots are complete, the buffer the next block's go to is
    // no longer read
    __syncthreads();
    float f[8];
    const bool ok = cube_corners<STORAGE>(m, s_nb[cur], threadIdx.x, f);
    prefetch_slots(m, b + gridDim.x, n, s_nb[cur ^ 1]);
    if (ok) mine += (uint32_t)cube_count(f);
  }
  __syncthreads();
  atomicAdd(&s_sum, mine);
  __syncthreads();
  if (threadIdx.x == 0) scratch[blockIdx.x] = s_sum;
}

// Pass 2 (one workgroup): exclusive offsets scratch[G + g] and the total.
__global__ __launch_bounds__(1024) void mesh_scan_kernel(uint32_t* scratch, int groups, uint32_t* count) {
  __shared__ uint32_t s_v[1024];
  const int t = threadIdx.x;
  const uint32_t x = t < groups ? scratch[t] : 0u;
  s_v[t] = x;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {  // inclusive Hillis-Steele scan
    const uint32_t y = t >= o ? s_v[t - o] : 0u;
    __syncthreads();
    s_v[t] += y;
    __syncthreads();
  }
  if (t < groups) scratch[groups + t] = s_v[t] - x;
  if (t == 1023) *count = s_v[1023];
}

// Pass 3: every workgroup walks the same blocks as in pass 1 and writes its
// triangles from its offset, threads in order within each block.
template <int STORAGE>
__global__ __launch_bounds__(kMeshThreads) void mesh_write_kernel(MapDev m, const uint32_t* scratch, int groups,
                                                                  float* tris, uint32_t cap) {
  __shared__ int s_nb[2][8];
  __shared__ uint32_t s_wave[kMeshThreads / 64];
  __shared__ uint32_t s_swave[kMeshThreads / 64];
  // the block's cubes that emit triangles, compacted in thread order: cube,
  // first output triangle, corner values
  __shared__ uint16_t s_cube[kMeshThreads];
  __shared__ uint32_t s_off[kMeshThreads];
  __shared__ float s_f[kMeshThreads][8];
  const uint32_t n = min(m.st->n_blocks, m.max_blocks);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t base = scratch[groups + blockIdx.x];
  const float s = m.s;
  prefetch_slots(m, blockIdx.x, n, s_nb[0]);
  int cur = 0;
  for (uint32_t b = blockIdx.x; b < n; b += gridDim.x, cur ^= 1) {
    int bx, by, bz;
    unpack_key(m.block_keys[b], bx, by, bz);
    // this block's slots are complete; the previous block's LDS lists and
    // the buffer the next block's slots go to are no longer read
    __syncthreads();
    float f[8];
    const bool ok = cube_corners<STORAGE>(m, s_nb[cur], threadIdx.x, f);
    prefetch_slots(m, b + gridDim.x, n, s_nb[cur ^ 1]);
    const uint32_t cnt = ok ? (uint32_t)cube_count(f) : 0u;
    // exclusive prefix over the workgroup in thread order
    uint32_t inc = cnt;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const uint32_t y = __shfl_up(inc, o);
      if (lane >= o) inc += y;
    }
    const unsigned long long sb = __ballot(cnt != 0u);
    if (lane == 63) s_wave[wave] = inc;
    if (lane == 0) s_swave[wave] = (uint32_t)__popcll(sb);
    __syncthreads();
    uint32_t before = 0, total = 0, sbefore = 0, stotal = 0;
#pragma unroll
    for (int w = 0; w < kMeshThreads / 64; ++w) {
      const uint32_t tw = s_wave[w], sw = s_swave[w];
      before += w < wave ? tw : 0u;
      total += tw;
      sbefore += w < wave ? sw : 0u;
      stotal += sw;
    }
    // The cubes that emit triangles are packed in thread order, so their
    // triangles are written by consecutive threads at the same positions (a
    // block has tens of such cubes, spread over all its wavefronts).
    if (cnt) {
      const uint32_t pos = sbefore + __builtin_amdgcn_mbcnt_hi((uint32_t)(sb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)sb, 0u));
      s_cube[pos] = (uint16_t)threadIdx.x;
      s_off[pos] = base + before + inc - cnt;
#pragma unroll
      for (int k = 0; k < 8; ++k) s_f[pos][k] = f[k];
    }
    __syncthreads();
    if (threadIdx.x < stotal) {
      const int l = s_cube[threadIdx.x];
      const int v[3] = {8 * bx + (l & 7), 8 * by + ((l >> 3) & 7), 8 * bz + (l >> 6)};
      float fc[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) fc[k] = s_f[threadIdx.x][k];
      MeshOut out{tris, cap, s_off[threadIdx.x]};
      cube_write(fc, v, s, out);
    }
    base += total;
  }
}

constexpr int kMeshGroups = kMeshScratch;

void launch_mesh(const MapDev& m, int storage, float* tris, uint32_t cap, uint32_t* count, hipStream_t s) {
  if (storage == RF_STORAGE_FP32) {
    mesh_count_kernel<RF_STORAGE_FP32><<<kMeshGroups, kMeshThreads, 0, s>>>(m, m.mesh_scratch);
    mesh_scan_kernel<<<1, 1024, 0, s>>>(m.mesh_scratch, kMeshGroups, count);
    mesh_write_kernel<RF_STORAGE_FP32><<<kMeshGroups, kMeshThreads, 0, s>>>(m, m.mesh_scratch, kMeshGroups, tris, cap);
  } else {
    mesh_count_kernel<RF_STORAGE_FP16_U8><<<kMeshGroups, kMeshThreads, 0, s>>>(m, m.mesh_scratch);
    mesh_scan_kernel<<<1, 1024, 0, s>>>(m.mesh_scratch, kMeshGroups, count);
    mesh_write_kernel<RF_STORAGE_FP16_U8><<<kMeshGroups, kMeshThreads, 0, s>>>(m, m.mesh_scratch, kMeshGroups, tris,
                                                                              cap);
  }
}

}  // namespace rf
