// blocks.hip -- block min/max build and TF-dependent block occupancy (gfx950).
//
// The paper decomposes the volume into fixed-size blocks (smaller at the far
// faces) that overlap by the voxels a cubic stencil reads, and drops blocks
// with nothing visible (Section 2, block decomposition, Fig. 3, "Pros" (a),
// (b)).  Here a block is the cell range [bE, bE+E) per axis; its footprint
// [bE-1, bE+E+1] (clamped) is every voxel a tricubic sample with its cell in
// the block can read, and the per-block (min, max) over that footprint,
// together with the TF, decides whether the block can hold a visible sample.
#include "vr_internal.h"

namespace vr {

// One workgroup per row of blocks (by, bz): the x-rows of its footprint,
// [16 by - 1, 16 by + 17] x [16 bz - 1, 16 bz + 17] (clamped), are streamed
// once; the eight wavefronts take every eighth row, four rows per trip (their
// loads in flight together).  In a pass over 32 blocks of x, a lane holds the
// E/2 voxels of half a block: even lane 2i the low half of block i of the
// pass plus the voxel before it, odd lane 2i + 1 the high half plus the two
// after it (x clamped to the row, which duplicates edge voxels and leaves
// min and max unchanged), so the block's footprint along x is the pair's
// union, combined with one lane swap.  The even lane keeps the running (min,
// max) over the rows; the wavefronts are combined in LDS at the end of the
// pass.  WIDE (E = 16, rows of a multiple of 8 voxels, 16-byte aligned data):
// a lane's half block is one or two 16-byte loads; 16-bit voxels take
// k_block_minmax_pk16 (packed integer min/max, z streaming) below.
constexpr int kMinmaxHalf = 8;   // voxels per lane per row in one trip: half of a 16-voxel block
constexpr int kMinmaxRows = 4;   // rows per wavefront trip (2 to 8 measured; 8 slower)
constexpr int kMinmaxThreads = 512;  // eight wavefronts: more rows in flight per row of blocks

template <typename T>
__device__ inline void half_block_range(const T *row, int xa, int half, int nx, bool hi, float &mn, float &mx) {
  // the footprint's apron: one voxel before the block, two after it
  // (lanes whose block lies past the grid in the last pass clamp too: every
  // index stays inside the row)
  const float a0 = (float)row[hi ? min(xa + half, nx - 1) : min(max(xa - 1, 0), nx - 1)];
  const float a1 = (float)row[hi ? min(xa + half + 1, nx - 1) : min(xa, nx - 1)];
  mn = fminf(mn, fminf(a0, a1));
  mx = fmaxf(mx, fmaxf(a0, a1));
  for (int i0 = 0; i0 < half; i0 += kMinmaxHalf) {  // one trip for E <= 16
    float a[kMinmaxHalf];
#pragma unroll
    for (int i = 0; i < kMinmaxHalf; ++i) a[i] = (float)row[min(xa + min(i0 + i, half - 1), nx - 1)];
#pragma unroll
    for (int i = 0; i < kMinmaxHalf; ++i) {
      mn = fminf(mn, a[i]);
      mx = fmaxf(mx, a[i]);
    }
  }
}

// WIDE: E = 16, rows of a multiple of 8 voxels, 16-byte aligned.  A lane's
// half block (xa a multiple of 8) is one 16-byte load (two for fp32); past
// the row's end the row's last 8 voxels stand in (they lie in the last
// block's footprint).  The apron comes from the neighbouring lanes' loads
// (the last voxel of lane - 1, the first two of lane + 1); only the lanes at
// the ends of a pass load theirs (lane 0 the voxel before the pass, lane 63
// the two after it, clamped to the row).
template <typename T>
__device__ inline void half_block_range_wide(const T *row, int xa, int nx, int lane, bool first_pass, float &mn,
                                             float &mx) {
  const T *p = row + min(xa, nx - kMinmaxHalf);
  float a[kMinmaxHalf];
  if constexpr (sizeof(T) == 2) {
    const uint4 q = *reinterpret_cast<const uint4 *>(p);
    const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const uint16_t lo = (uint16_t)(w[i] & 0xffffu), h = (uint16_t)(w[i] >> 16);
      a[2 * i] = (float)*reinterpret_cast<const T *>(&lo);
      a[2 * i + 1] = (float)*reinterpret_cast<const T *>(&h);
    }
  } else {
    const float4 q0 = reinterpret_cast<const float4 *>(p)[0], q1 = reinterpret_cast<const float4 *>(p)[1];
    a[0] = q0.x; a[1] = q0.y; a[2] = q0.z; a[3] = q0.w;
    a[4] = q1.x; a[5] = q1.y; a[6] = q1.z; a[7] = q1.w;
  }
  const float left = __shfl_up(a[kMinmaxHalf - 1], 1, kWaveSize);
  const float right0 = __shfl_down(a[0], 1, kWaveSize), right1 = __shfl_down(a[1], 1, kWaveSize);
  float ap0, ap1;
  if (lane & 1) {
    if (lane == kWaveSize - 1) {
      ap0 = (float)row[min(xa + kMinmaxHalf, nx - 1)];
      ap1 = (float)row[min(xa + kMinmaxHalf + 1, nx - 1)];
    } else {
      ap0 = right0;
      ap1 = right1;
    }
  } else {
    ap0 = lane == 0 ? (first_pass ? a[0] : (float)row[min(max(xa - 1, 0), nx - 1)]) : left;
    ap1 = ap0;
  }
  mn = fminf(mn, fminf(ap0, ap1));
  mx = fmaxf(mx, fmaxf(ap0, ap1));
#pragma unroll
  for (int i = 0; i < kMinmaxHalf; ++i) {
    mn = fminf(mn, a[i]);
    mx = fmaxf(mx, a[i]);
  }
}

// WIDE for 16-bit voxels: the running (min, max) of a lane stay packed 16-bit
// integers (two per register, v_pk_min / v_pk_max over the four dwords of a
// load), exact, and become floats once per pass; the apron dwords come from
// the neighbouring lanes (the last dword of lane - 1, of which the high half
// is the voxel before the block; the first dword of lane + 1, both halves
// after it).
typedef short s16x2 __attribute__((ext_vector_type(2)));
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

template <typename T>
struct Packed16;
template <>
struct Packed16<int16_t> {
  typedef s16x2 V;
  static constexpr short kLo = -32768, kHi = 32767;
};
template <>
struct Packed16<uint16_t> {
  typedef u16x2 V;
  static constexpr unsigned short kLo = 0, kHi = 65535;
};

template <typename T>
__device__ inline void half_block_range_pk16(const T *row, int xa, int nx, int lane, bool first_pass,
                                             typename Packed16<T>::V &mn, typename Packed16<T>::V &mx) {
  typedef typename Packed16<T>::V V;
  const uint4 q = *reinterpret_cast<const uint4 *>(row + min(xa, nx - kMinmaxHalf));
  const V w0 = __builtin_bit_cast(V, q.x), w1 = __builtin_bit_cast(V, q.y);
  const V w2 = __builtin_bit_cast(V, q.z), w3 = __builtin_bit_cast(V, q.w);
  mn = __builtin_elementwise_min(mn, __builtin_elementwise_min(__builtin_elementwise_min(w0, w1),
                                                               __builtin_elementwise_min(w2, w3)));
  mx = __builtin_elementwise_max(mx, __builtin_elementwise_max(__builtin_elementwise_max(w0, w1),
                                                               __builtin_elementwise_max(w2, w3)));
  const uint32_t left = (uint32_t)__shfl_up((int)q.w, 1, kWaveSize);
  const uint32_t right = (uint32_t)__shfl_down((int)q.x, 1, kWaveSize);
  uint32_t ap;
  if (lane & 1) {
    if (lane == kWaveSize - 1) {
      const uint32_t a0 = (uint16_t)row[min(xa + kMinmaxHalf, nx - 1)], a1 = (uint16_t)row[min(xa + kMinmaxHalf + 1, nx - 1)];
      ap = a0 | (a1 << 16);
    } else {
      ap = right;
    }
  } else {
    uint32_t v;  // the voxel before the block, in the low half
    if (lane == 0)
      v = first_pass ? (q.x & 0xffffu) : (uint16_t)row[min(max(xa - 1, 0), nx - 1)];
    else
      v = left >> 16;
    ap = v | (v << 16);
  }
  mn = __builtin_elementwise_min(mn, __builtin_bit_cast(V, ap));
  mx = __builtin_elementwise_max(mx, __builtin_bit_cast(V, ap));
}

// One workgroup per row of blocks in x and BZ consecutive blocks in z: the
// x-rows of the footprint are streamed in z order, each read once, and a row
// adds to the one or two blocks in z whose footprint holds it (z in
// [16 b - 1, 16 b + 17]): rows shared by vertically neighbouring blocks are
// not read again.  (With BZ = 1 every block row reads its own footprint, as
// k_block_minmax does; the launch takes BZ = 4 when that still leaves about
// four workgroups per CU.)
template <typename T, int BZ>
__global__ __launch_bounds__(kMinmaxThreads) void k_block_minmax_pk16(const VolConst v, float2 *out) {
  typedef typename Packed16<T>::V V;
  constexpr int kWaves = kMinmaxThreads / kWaveSize;
  constexpr int E = 2 * kMinmaxHalf;
  __shared__ float smin[BZ][kWaves][kWaveSize / 2], smax[BZ][kWaves][kWaveSize / 2];
  // XCD-aware: workgroup i runs on XCD i mod 8; each XCD takes a contiguous
  // run of items, neighbouring rows of blocks in y side by side
  const int nchunks = (v.nbz + BZ - 1) / BZ;
  const int nitems = v.nby * nchunks, per_xcd = (nitems + kXcds - 1) / kXcds;
  const int q = (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds);
  if (q >= nitems) return;
  const int by = q % v.nby, bz0 = (q / v.nby) * BZ, nbz = min(BZ, v.nbz - bz0);
  const int y0 = max(by * E - 1, 0), y1 = min(by * E + E + 1, v.ny - 1);
  const int z0 = max(bz0 * E - 1, 0), z1 = min((bz0 + nbz) * E + 1, v.nz - 1);
  const int ny = y1 - y0 + 1, rows = ny * (z1 - z0 + 1);
  // the wavefront index, as a uniform value: the row walk below stays scalar
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / kWaveSize));
  const int lane = threadIdx.x % kWaveSize;
  const T *base = reinterpret_cast<const T *>(v.data);
  constexpr int per_pass = kWaveSize / 2;  // blocks per pass
  for (int bx0 = 0; bx0 < v.nbx; bx0 += per_pass) {
    const int bx = bx0 + lane / 2;
    const bool hi = lane & 1;
    const int xa = bx * E + (hi ? kMinmaxHalf : 0);
    V mn[BZ], mx[BZ];
#pragma unroll
    for (int j = 0; j < BZ; ++j) {
      mn[j] = V{Packed16<T>::kHi, Packed16<T>::kHi};
      mx[j] = V{Packed16<T>::kLo, Packed16<T>::kLo};
    }
    // footprint row r = (y - y0) + ny (z - z0), walked by increments (no
    // division per row); rows past the last repeat it, which changes nothing
    int r = wave, y = y0 + wave % ny, z = z0 + wave / ny;
    while (r < rows) {
#pragma unroll
      for (int u = 0; u < kMinmaxRows; ++u) {
        const bool in = r < rows;
        const int yy = in ? y : y1, zz = in ? z : z1;
        const T *row = base + ((size_t)zz * (size_t)v.ny + (size_t)yy) * (size_t)v.nx;
        V rmn = V{Packed16<T>::kHi, Packed16<T>::kHi}, rmx = V{Packed16<T>::kLo, Packed16<T>::kLo};
        half_block_range_pk16<T>(row, xa, v.nx, lane, bx0 == 0, rmn, rmx);
        if constexpr (BZ == 1) {
          mn[0] = __builtin_elementwise_min(mn[0], rmn);
          mx[0] = __builtin_elementwise_max(mx[0], rmx);
        } else {
          // the blocks in z whose footprint holds row zz (one, or two at a
          // boundary), relative to this item's first
          const int jhi = (zz + 1) / E - bz0, jlo = (zz + E - 2) / E - 1 - bz0;
#pragma unroll
          for (int j = 0; j < BZ; ++j)
            if ((j == jhi || j == jlo) && j < nbz) {  // uniform
              mn[j] = __builtin_elementwise_min(mn[j], rmn);
              mx[j] = __builtin_elementwise_max(mx[j], rmx);
            }
        }
        r += kWaves;
        y += kWaves;
        while (y > y1) {
          y -= ny;
          ++z;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < BZ; ++j) {
      float fmn = (float)min(mn[j].x, mn[j].y), fmx = (float)max(mx[j].x, mx[j].y);
      fmn = fminf(fmn, __shfl_xor(fmn, 1, kWaveSize));
      fmx = fmaxf(fmx, __shfl_xor(fmx, 1, kWaveSize));
      if (!hi) {
        smin[j][wave][lane / 2] = fmn;
        smax[j][wave][lane / 2] = fmx;
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < per_pass * nbz; t += kMinmaxThreads) {
      const int j = t / per_pass, i = t % per_pass, b = bx0 + i;
      float m0 = smin[j][0][i], m1 = smax[j][0][i];
#pragma unroll
      for (int w = 1; w < kWaves; ++w) {
        m0 = fminf(m0, smin[j][w][i]);
        m1 = fmaxf(m1, smax[j][w][i]);
      }
      if (b < v.nbx) out[((int64_t)(bz0 + j) * v.nby + by) * v.nbx + b] = make_float2(m0, m1);
    }
    __syncthreads();
  }
}

template <typename T, bool WIDE>
__global__ __launch_bounds__(kMinmaxThreads) void k_block_minmax(const VolConst v, float2 *out) {
  constexpr int kWaves = kMinmaxThreads / kWaveSize;
  __shared__ float smin[kWaves][kWaveSize / 2], smax[kWaves][kWaveSize / 2];
  // XCD-aware: the hardware hands workgroup i to XCD i mod 8; each XCD takes
  // a contiguous run of rows of blocks, so the footprint rows neighbouring
  // rows of blocks share are read through the same L2
  const int nrows = v.nby * v.nbz, per_xcd = (nrows + kXcds - 1) / kXcds;
  const int q = (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds);
  if (q >= nrows) return;  // uniform: padding of the last XCD's run
  const int by = q % v.nby, bz = q / v.nby;
  const int E = v.edge, half = E / 2;
  const int y0 = max(by * E - 1, 0), y1 = min(by * E + E + 1, v.ny - 1);
  const int z0 = max(bz * E - 1, 0), z1 = min(bz * E + E + 1, v.nz - 1);
  const int ny = y1 - y0 + 1, rows = ny * (z1 - z0 + 1);
  const int wave = threadIdx.x / kWaveSize, lane = threadIdx.x % kWaveSize;
  const T *base = reinterpret_cast<const T *>(v.data);
  const int per_pass = kWaveSize / 2;  // blocks per pass
  for (int bx0 = 0; bx0 < v.nbx; bx0 += per_pass) {
    const int bx = bx0 + lane / 2;          // this lane's block
    const bool hi = lane & 1;
    const int xa = bx * E + (hi ? half : 0);  // first voxel of its half
    float mn = INFINITY, mx = -INFINITY;
    for (int r0 = wave; r0 < rows; r0 += kWaves * kMinmaxRows) {
#pragma unroll
      for (int u = 0; u < kMinmaxRows; ++u) {
        const int r = min(r0 + u * kWaves, rows - 1);  // a repeated last row changes nothing
        const int y = y0 + r % ny, z = z0 + r / ny;
        const T *row = base + ((size_t)z * (size_t)v.ny + (size_t)y) * (size_t)v.nx;
        if constexpr (WIDE)
          half_block_range_wide<T>(row, xa, v.nx, lane, bx0 == 0, mn, mx);
        else
          half_block_range<T>(row, xa, half, v.nx, hi, mn, mx);
      }
    }
    // the pair's union: the even lane takes its odd neighbour's range
    mn = fminf(mn, __shfl_xor(mn, 1, kWaveSize));
    mx = fmaxf(mx, __shfl_xor(mx, 1, kWaveSize));
    if (!hi) {
      smin[wave][lane / 2] = mn;
      smax[wave][lane / 2] = mx;
    }
    __syncthreads();
    if (threadIdx.x < per_pass) {
      const int b = bx0 + threadIdx.x;
      float m0 = smin[0][threadIdx.x], m1 = smax[0][threadIdx.x];
#pragma unroll
      for (int w = 1; w < kWaves; ++w) {
        m0 = fminf(m0, smin[w][threadIdx.x]);
        m1 = fmaxf(m1, smax[w][threadIdx.x]);
      }
      if (b < v.nbx) out[((int64_t)bz * v.nby + by) * v.nbx + b] = make_float2(m0, m1);
    }
    __syncthreads();
  }
}

// Blocks in z per workgroup of the 16-bit kernel: four when that leaves at
// least kMinmaxStreamItems workgroups (four per CU), else one.
constexpr int kMinmaxStreamItems = 1024;

template <typename T>
static void launch_minmax_pk16(const VolConst &v, float2 *out, hipStream_t s) {
  const int64_t items4 = (int64_t)v.nby * ((v.nbz + 3) / 4);
  if (items4 >= kMinmaxStreamItems) {
    const unsigned grid = (unsigned)((items4 + kXcds - 1) / kXcds * kXcds);
    hipLaunchKernelGGL((k_block_minmax_pk16<T, 4>), dim3(grid), dim3(kMinmaxThreads), 0, s, v, out);
  } else {
    const unsigned grid = (unsigned)(((int64_t)v.nby * v.nbz + kXcds - 1) / kXcds * kXcds);
    hipLaunchKernelGGL((k_block_minmax_pk16<T, 1>), dim3(grid), dim3(kMinmaxThreads), 0, s, v, out);
  }
}

hipError_t launch_block_minmax(const VolConst &v, float2 *out, hipStream_t s) {
  const unsigned grid = (unsigned)(((int64_t)v.nby * v.nbz + kXcds - 1) / kXcds * kXcds);
  const bool wide = v.edge == 2 * kMinmaxHalf && v.nx % kMinmaxHalf == 0 &&
                    (reinterpret_cast<uintptr_t>(v.data) & 15u) == 0;
  switch (v.dtype) {
  case kU16:
    if (wide) launch_minmax_pk16<uint16_t>(v, out, s);
    else hipLaunchKernelGGL((k_block_minmax<uint16_t, false>), dim3(grid), dim3(kMinmaxThreads), 0, s, v, out);
    break;
  case kI16:
    if (wide) launch_minmax_pk16<int16_t>(v, out, s);
    else hipLaunchKernelGGL((k_block_minmax<int16_t, false>), dim3(grid), dim3(kMinmaxThreads), 0, s, v, out);
    break;
  case kF32:
    if (wide) hipLaunchKernelGGL((k_block_minmax<float, true>), dim3(grid), dim3(kMinmaxThreads), 0, s, v, out);
    else hipLaunchKernelGGL((k_block_minmax<float, false>), dim3(grid), dim3(kMinmaxThreads), 0, s, v, out);
    break;
  default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// One thread per block; the TF and its prefix counts sit in LDS.  The same
// decision (range_occupied) is taken on the fly by the render kernels.
__global__ __launch_bounds__(kWgSize) void k_block_occupancy(const VolConst v, const TfConst tf, uint8_t *occ) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  TfShared s = carve_tf(lds, tf.K);
  load_tf(s, tf);
  const int64_t nb = (int64_t)v.nbx * v.nby * v.nbz;
  const int64_t b = (int64_t)blockIdx.x * kWgSize + threadIdx.x;
  if (b < nb) occ[b] = block_occupied(v, s, tf, (int)b) ? 1 : 0;
}

hipError_t launch_block_occupancy(const VolConst &v, const TfConst &tf, uint8_t *occ, hipStream_t s) {
  int64_t nb = (int64_t)v.nbx * v.nby * v.nbz;
  unsigned grid = (unsigned)((nb + kWgSize - 1) / kWgSize);
  hipLaunchKernelGGL(k_block_occupancy, dim3(grid), dim3(kWgSize), tf_lds_bytes(tf.K), s, v, tf, occ);
  return hipGetLastError();
}

// One thread per block, one ballot per 64 blocks; bits past the last block
// are zero.
__global__ __launch_bounds__(kWgSize) void k_occupancy_bits(const VolConst v, const TfConst tf, uint32_t *bits) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  TfShared s = carve_tf(lds, tf.K);
  load_tf(s, tf);
  const int64_t nb = (int64_t)v.nbx * v.nby * v.nbz;
  const int64_t b = (int64_t)blockIdx.x * kWgSize + threadIdx.x;
  const unsigned long long m = __ballot(b < nb && block_occupied(v, s, tf, (int)b));
  const int lane = threadIdx.x % kWaveSize;
  if ((lane == 0 || lane == 32) && b < nb) bits[b >> 5] = lane == 0 ? (uint32_t)m : (uint32_t)(m >> 32);
}

hipError_t launch_occupancy_bits(const VolConst &v, const TfConst &tf, uint32_t *bits, hipStream_t s) {
  VolConst vm = v;
  vm.occ = nullptr;  // decide from minmax
  const int64_t nb = (int64_t)v.nbx * v.nby * v.nbz;
  const unsigned grid = (unsigned)((nb + kWgSize - 1) / kWgSize);
  hipLaunchKernelGGL(k_occupancy_bits, dim3(grid), dim3(kWgSize), tf_lds_bytes(tf.K), s, vm, tf, bits);
  return hipGetLastError();
}

// Both planes in one launch: the occupancy bits (plane 0, as k_occupancy_bits)
// and the radius plane after them: 2 bits per block (16 blocks a word), for
// an empty block b the largest r <= kEmptyRadiusMax such that every block
// within Chebyshev distance r of b is empty (outside the grid counts as
// empty), 0 for occupied blocks.  The blocks around a workgroup's
// kPlanesThreads consecutive blocks lie within empty_reach bit positions of
// them: the workgroup decides the occupancy of that window itself (from
// min/max and the TF in LDS), writes plane 0 for its own blocks, and reads
// each x-row of a neighbourhood as one bit field of at most 2R + 1 bits.
// Workgroups of 1024 threads: the window (three planes of blocks on either
// side) is shared by four times the blocks of a 256-thread workgroup, and
// each wavefront walks a quarter of the loads one after another (C1: 21 us
// with 256 threads).
constexpr int kPlanesThreads = 1024;
__host__ __device__ inline int64_t empty_reach(const VolConst &v) {
  return kEmptyRadiusMax * (1 + (int64_t)v.nbx + (int64_t)v.nbx * v.nby);
}
__host__ __device__ inline int64_t empty_window_words(const VolConst &v) {
  return (kPlanesThreads + 2 * empty_reach(v)) / 32 + 2;
}
__host__ __device__ inline uint32_t planes_lds_bytes(const VolConst &v, int K) {
  return ((tf_lds_bytes(K) + 15u) & ~15u) + (uint32_t)empty_window_words(v) * 4u;
}

// Bits 0..15 of x moved to the even positions 0, 2, .., 30.
__device__ inline uint32_t spread16(uint32_t x) {
  x &= 0xffffu;
  x = (x | (x << 8)) & 0x00ff00ffu;
  x = (x | (x << 4)) & 0x0f0f0f0fu;
  x = (x | (x << 2)) & 0x33333333u;
  x = (x | (x << 1)) & 0x55555555u;
  return x;
}

__global__ __launch_bounds__(kPlanesThreads) void k_occupancy_planes(const VolConst v, const TfConst tf, uint32_t *bits) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  TfShared s = carve_tf(lds, tf.K);
  uint32_t *win = reinterpret_cast<uint32_t *>(lds + ((tf_lds_bytes(tf.K) + 15u) & ~15u));
  load_tf<kPlanesThreads>(s, tf);  // ends with a barrier
  const int64_t nb = (int64_t)v.nbx * v.nby * v.nbz;
  const int64_t words = (nb + 31) / 32;
  const int64_t b0 = (int64_t)blockIdx.x * kPlanesThreads;
  const int64_t w0 = max(b0 - empty_reach(v), (int64_t)0) >> 5;
  const int64_t nw = empty_window_words(v);
  // window occupancy: each wavefront decides 64 blocks (two words) at a time
  const int lane = threadIdx.x % kWaveSize, wave = threadIdx.x / kWaveSize;
  for (int64_t j = 2 * wave; j < nw; j += 2 * (kPlanesThreads / kWaveSize)) {
    const int64_t q = 32 * (w0 + j) + lane;
    const unsigned long long m = __ballot(q < nb && block_occupied(v, s, tf, (int)q));
    if (lane == 0) win[j] = (uint32_t)m;
    if (lane == 32 && j + 1 < nw) win[j + 1] = (uint32_t)(m >> 32);
  }
  __syncthreads();
  if (threadIdx.x < kPlanesThreads / 32) {  // plane 0 of this workgroup's blocks
    const int64_t w = (b0 >> 5) + threadIdx.x;
    if (w < words) bits[w] = win[w - w0];
  }
  const int64_t b = b0 + threadIdx.x;
  int rad = 0;
  if (b < nb) {
    const int bx = (int)(b % v.nbx), by = (int)((b / v.nbx) % v.nby), bz = (int)(b / ((int64_t)v.nbx * v.nby));
    constexpr int R = kEmptyRadiusMax;
    const int lx = max(bx - R, 0), hx = min(bx + R, v.nbx - 1), c = bx - lx, n = hx - lx + 1;
    int near = R + 1;  // smallest Chebyshev distance of an occupied block, capped at R + 1
    for (int dz = -R; dz <= R; ++dz)
      for (int dy = -R; dy <= R; ++dy) {
        const int y = by + dy, z = bz + dz;
        if (y < 0 || z < 0 || y >= v.nby || z >= v.nbz) continue;
        // bits lx .. hx of row (y, z)
        const int64_t q = lx + (int64_t)v.nbx * (y + (int64_t)v.nby * z) - 32 * w0;
        const int64_t w = q >> 5;
        const int off = (int)(q & 31);
        const uint64_t pair = (uint64_t)win[w] | (w + 1 < nw ? (uint64_t)win[w + 1] << 32 : 0ull);
        const uint32_t field = (uint32_t)(pair >> off) & ((1u << n) - 1u);
        if (!field) continue;
        int dx = R;
        for (int t = 0; t < R; ++t) {  // nearest set bit to position c
          const int lo = max(c - t, 0), hi = min(c + t, n - 1);
          if (field & (((1u << (hi - lo + 1)) - 1u) << lo)) {
            dx = t;
            break;
          }
        }
        near = min(near, max(max(abs(dy), abs(dz)), dx));
      }
    rad = near - 1 < 0 ? 0 : near - 1;
  }
  const unsigned long long lo = __ballot(rad & 1), hi = __ballot(rad & 2);
  const int64_t rw = words + (b >> 4);
  if ((lane & 15) == 0 && b < nb)
    bits[rw] = spread16((uint32_t)(lo >> lane)) | (spread16((uint32_t)(hi >> lane)) << 1);
}

bool occupancy_planes_fit(const VolConst &v, int K) { return planes_lds_bytes(v, K) <= max_lds_per_workgroup(); }

hipError_t launch_occupancy_planes(const VolConst &v, const TfConst &tf, uint32_t *bits, hipStream_t s) {
  if (!occupancy_planes_fit(v, tf.K)) return hipErrorInvalidValue;  // the caller leaps block by block
  VolConst vm = v;
  vm.occ = nullptr;  // decide from min/max
  const int64_t nb = (int64_t)v.nbx * v.nby * v.nbz;
  const uint32_t lds = planes_lds_bytes(v, tf.K);
  const unsigned grid = (unsigned)((nb + kPlanesThreads - 1) / kPlanesThreads);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_occupancy_planes),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_occupancy_planes, dim3(grid), dim3(kPlanesThreads), lds, s, vm, tf, bits);
  return hipGetLastError();
}

// Widened block ranges [lo - w (hi - lo), hi + w (hi - lo)] (fused, fp32).
__global__ __launch_bounds__(kWgSize) void k_widen_minmax(const float2 *in, float2 *out, int64_t n, float w) {
  const int64_t i = (int64_t)blockIdx.x * kWgSize + threadIdx.x;
  if (i < n) {
    const float2 m = in[i];
    const float d = m.y - m.x;
    out[i] = make_float2(fmaf(-w, d, m.x), fmaf(w, d, m.y));
  }
}

hipError_t launch_widen_minmax(const float2 *in, float2 *out, int64_t n, float w, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_widen_minmax, dim3((unsigned)((n + kWgSize - 1) / kWgSize)), dim3(kWgSize), 0, s, in, out, n, w);
  return hipGetLastError();
}

__global__ __launch_bounds__(kWgSize) void k_fill_zero(float *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kWgSize + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWgSize) p[i] = 0.0f;
}

hipError_t launch_fill_zero(float *p, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  int64_t g = (n + kWgSize - 1) / kWgSize;
  if (g > 65536) g = 65536;
  hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)g), dim3(kWgSize), 0, s, p, n);
  return hipGetLastError();
}

}  // namespace vr

namespace vr {

// Interpolating cubic B-spline prefilter, one axis: every line solves
// (c[i-1] + 4 c[i] + c[i+1]) / 6 = v[i] with c[-1] = c[0], c[n] = c[n-1]
// (diagonal 5 in the end rows).  The elimination's pivots depend only on the
// line length, so they come precomputed (inv_piv[i] = 1 / pivot i, sup[i] the
// eliminated super-diagonal); a thread sweeps one line forward and back, in
// place.  Lines along y and z are coalesced across a wavefront's lanes.
__global__ __launch_bounds__(kWgSize) void k_prefilter_axis(float *vol, int nx, int ny, int nz, int axis,
                                                            const float *inv_piv, const float *sup) {
  const int64_t line = (int64_t)blockIdx.x * kWgSize + threadIdx.x;
  int64_t base, stride;
  int n;
  if (axis == 0) {
    if (line >= (int64_t)ny * nz) return;
    base = line * nx;
    stride = 1;
    n = nx;
  } else if (axis == 1) {
    if (line >= (int64_t)nx * nz) return;
    const int64_t x = line % nx, z = line / nx;
    base = z * (int64_t)nx * ny + x;
    stride = nx;
    n = ny;
  } else {
    if (line >= (int64_t)nx * ny) return;
    base = line;
    stride = (int64_t)nx * ny;
    n = nz;
  }
  if (n == 1) return;
  float *p = vol + base;
  float prev = 6.0f * p[0] * inv_piv[0];
  p[0] = prev;
  for (int i = 1; i < n; ++i) {
    prev = (6.0f * p[(int64_t)i * stride] - prev) * inv_piv[i];
    p[(int64_t)i * stride] = prev;
  }
  float next = prev;
  for (int i = n - 2; i >= 0; --i) {
    next = p[(int64_t)i * stride] - sup[i] * next;
    p[(int64_t)i * stride] = next;
  }
}

// Copy a volume of any dtype into fp32.
template <int DT>
__global__ __launch_bounds__(kWgSize) void k_to_f32(const void *src, float *dst, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * kWgSize + threadIdx.x; i < n; i += (int64_t)gridDim.x * kWgSize) {
    if (DT == kF32)
      dst[i] = reinterpret_cast<const float *>(src)[i];
    else if (DT == kI16)
      dst[i] = (float)reinterpret_cast<const int16_t *>(src)[i];
    else
      dst[i] = (float)reinterpret_cast<const uint16_t *>(src)[i];
  }
}

hipError_t launch_prefilter(const VolConst &v, float *out, const float *coef, hipStream_t s) {
  const int64_t n = (int64_t)v.nx * v.ny * v.nz;
  int64_t g = (n + kWgSize - 1) / kWgSize;
  if (g > 65536) g = 65536;
  switch (v.dtype) {
  case kU16: hipLaunchKernelGGL(k_to_f32<kU16>, dim3((unsigned)g), dim3(kWgSize), 0, s, v.data, out, n); break;
  case kI16: hipLaunchKernelGGL(k_to_f32<kI16>, dim3((unsigned)g), dim3(kWgSize), 0, s, v.data, out, n); break;
  default: hipLaunchKernelGGL(k_to_f32<kF32>, dim3((unsigned)g), dim3(kWgSize), 0, s, v.data, out, n); break;
  }
  const int dims[3] = {v.nx, v.ny, v.nz};
  int64_t off = 0;
  for (int axis = 0; axis < 3; ++axis) {
    const int64_t lines = n / dims[axis];
    hipLaunchKernelGGL(k_prefilter_axis, dim3((unsigned)((lines + kWgSize - 1) / kWgSize)), dim3(kWgSize), 0, s, out,
                       v.nx, v.ny, v.nz, axis, coef + off, coef + off + dims[axis]);
    off += 2 * (int64_t)dims[axis];
  }
  return hipGetLastError();
}

}  // namespace vr
