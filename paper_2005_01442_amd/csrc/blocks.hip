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

template <typename T>
__device__ inline float load_voxel(const void *p, uint32_t i) {
  return (float)reinterpret_cast<const T *>(p)[i];
}

// One workgroup per block streams its footprint and reduces it.
template <typename T>
__global__ __launch_bounds__(kWgSize) void k_block_minmax(const VolConst v, float2 *out) {
  __shared__ float smin[kWgSize / kWaveSize], smax[kWgSize / kWaveSize];
  const int64_t b = blockIdx.x;
  const int bx = (int)(b % v.nbx), by = (int)((b / v.nbx) % v.nby), bz = (int)(b / ((int64_t)v.nbx * v.nby));
  const int E = v.edge;
  const int x0 = max(bx * E - 1, 0), x1 = min(bx * E + E + 1, v.nx - 1);
  const int y0 = max(by * E - 1, 0), y1 = min(by * E + E + 1, v.ny - 1);
  const int z0 = max(bz * E - 1, 0), z1 = min(bz * E + E + 1, v.nz - 1);
  const int ex = x1 - x0 + 1, ey = y1 - y0 + 1, ez = z1 - z0 + 1;
  const int count = ex * ey * ez;
  float mn = INFINITY, mx = -INFINITY;
  for (int i = threadIdx.x; i < count; i += kWgSize) {
    int x = x0 + i % ex, y = y0 + (i / ex) % ey, z = z0 + i / (ex * ey);
    uint32_t idx = ((uint32_t)z * (uint32_t)v.ny + (uint32_t)y) * (uint32_t)v.nx + (uint32_t)x;
    float a = load_voxel<T>(v.data, idx);
    mn = fminf(mn, a);
    mx = fmaxf(mx, a);
  }
  for (int off = 32; off > 0; off >>= 1) {
    mn = fminf(mn, __shfl_xor(mn, off, kWaveSize));
    mx = fmaxf(mx, __shfl_xor(mx, off, kWaveSize));
  }
  const int wave = threadIdx.x / kWaveSize, lane = threadIdx.x % kWaveSize;
  if (lane == 0) {
    smin[wave] = mn;
    smax[wave] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kWgSize / kWaveSize; ++w) {
      mn = fminf(mn, smin[w]);
      mx = fmaxf(mx, smax[w]);
    }
    out[b] = make_float2(mn, mx);
  }
}

hipError_t launch_block_minmax(const VolConst &v, float2 *out, hipStream_t s) {
  int64_t nb = (int64_t)v.nbx * v.nby * v.nbz;
  switch (v.dtype) {
  case kU16: hipLaunchKernelGGL(k_block_minmax<uint16_t>, dim3((unsigned)nb), dim3(kWgSize), 0, s, v, out); break;
  case kI16: hipLaunchKernelGGL(k_block_minmax<int16_t>, dim3((unsigned)nb), dim3(kWgSize), 0, s, v, out); break;
  case kF32: hipLaunchKernelGGL(k_block_minmax<float>, dim3((unsigned)nb), dim3(kWgSize), 0, s, v, out); break;
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
// empty), 0 for occupied blocks.  The blocks around a workgroup's 256
// consecutive blocks lie within empty_reach bit positions of them: the
// workgroup decides the occupancy of that window itself (from min/max and the
// TF in LDS), writes plane 0 for its own blocks, and reads each x-row of a
// neighbourhood as one bit field of at most 2R + 1 bits.
__host__ __device__ inline int64_t empty_reach(const VolConst &v) {
  return kEmptyRadiusMax * (1 + (int64_t)v.nbx + (int64_t)v.nbx * v.nby);
}
__host__ __device__ inline int64_t empty_window_words(const VolConst &v) {
  return (kWgSize + 2 * empty_reach(v)) / 32 + 2;
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

__global__ __launch_bounds__(kWgSize) void k_occupancy_planes(const VolConst v, const TfConst tf, uint32_t *bits) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  TfShared s = carve_tf(lds, tf.K);
  uint32_t *win = reinterpret_cast<uint32_t *>(lds + ((tf_lds_bytes(tf.K) + 15u) & ~15u));
  load_tf(s, tf);  // ends with a barrier
  const int64_t nb = (int64_t)v.nbx * v.nby * v.nbz;
  const int64_t words = (nb + 31) / 32;
  const int64_t b0 = (int64_t)blockIdx.x * kWgSize;
  const int64_t w0 = max(b0 - empty_reach(v), (int64_t)0) >> 5;
  const int64_t nw = empty_window_words(v);
  // window occupancy: each wavefront decides 64 blocks (two words) at a time
  const int lane = threadIdx.x % kWaveSize, wave = threadIdx.x / kWaveSize;
  for (int64_t j = 2 * wave; j < nw; j += 2 * (kWgSize / kWaveSize)) {
    const int64_t q = 32 * (w0 + j) + lane;
    const unsigned long long m = __ballot(q < nb && block_occupied(v, s, tf, (int)q));
    if (lane == 0) win[j] = (uint32_t)m;
    if (lane == 32 && j + 1 < nw) win[j + 1] = (uint32_t)(m >> 32);
  }
  __syncthreads();
  if (threadIdx.x < kWgSize / 32) {  // plane 0 of this workgroup's blocks
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
  const unsigned grid = (unsigned)((nb + kWgSize - 1) / kWgSize);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_occupancy_planes),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_occupancy_planes, dim3(grid), dim3(kWgSize), lds, s, vm, tf, bits);
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
