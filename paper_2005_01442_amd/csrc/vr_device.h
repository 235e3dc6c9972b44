// vr_device.h -- device building blocks of the gfx950 ray caster, shared by
// the forward, adjoint and serving kernels.
//
// Ray casting per Section 2 of the paper: one ray per pixel from the
// observer, fixed step, colour accumulated along the ray; the scalar is
// reconstructed with cubic-spline (tricubic) interpolation and classified
// after interpolation through the transfer function; rays stop once opaque and
// blocks with nothing visible are skipped (block decomposition, "Pros" (b)).
//
// Work layout: a wavefront owns an 8x8 pixel tile (one ray per lane), a
// workgroup of four wavefronts a 16x16 super-tile; the whole-image forward
// kernel marches each ray with a pair of lanes instead (8x4 rays per
// wavefront, half a super-tile per workgroup).  The transfer function and
// its non-zero-extinction bitmask live in LDS.  Volume taps are fetched with
// raw buffer loads (bounds-checked by the hardware): an x-row of four int16
// taps is one dwordx3 load plus two v_alignbit, an fp32 row one dwordx4 load.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace vr {

constexpr int kTileEdge = 8;          // pixels per wavefront tile edge
constexpr int kSuperEdge = 16;        // pixels per workgroup super-tile edge
constexpr int kWaveSize = 64;
constexpr int kWgSize = 256;
constexpr int kMaxTf = 1024;          // max TF nodes (LDS: 16 KiB table)
constexpr int kMaxCamsPerLaunch = 16; // cameras carried in kernel arguments
constexpr int kXcds = 8;              // MI355X: 8 accelerator complex dies
constexpr int kDefaultChunkEdge = 4;  // super-tiles per chunk edge (XCD mapping)
constexpr int kEmptyRadiusMax = 3;    // largest cube of empty blocks a leap crosses

enum Dtype : int32_t { kU16 = 0, kI16 = 1, kF32 = 2 };

// Wavefront-wide min / max over all 64 lanes (every lane active), returned as
// a uniform (scalar) value: a butterfly inside each row of 16 lanes through
// DPP lane permutations (quad_perm [1,0,3,2], quad_perm [2,3,0,1],
// row_half_mirror, row_mirror: VALU only, no LDS round trips), then the four
// row results combined on the scalar unit.
constexpr int kDppQuadSwap1 = 0xB1, kDppQuadSwap2 = 0x4E, kDppHalfMirror = 0x141, kDppMirror = 0x140;

__device__ inline int wave_min_i32(int x) {
  x = min(x, __builtin_amdgcn_mov_dpp(x, kDppQuadSwap1, 0xF, 0xF, false));
  x = min(x, __builtin_amdgcn_mov_dpp(x, kDppQuadSwap2, 0xF, 0xF, false));
  x = min(x, __builtin_amdgcn_mov_dpp(x, kDppHalfMirror, 0xF, 0xF, false));
  x = min(x, __builtin_amdgcn_mov_dpp(x, kDppMirror, 0xF, 0xF, false));
  return min(min(__builtin_amdgcn_readlane(x, 0), __builtin_amdgcn_readlane(x, 16)),
             min(__builtin_amdgcn_readlane(x, 32), __builtin_amdgcn_readlane(x, 48)));
}

__device__ inline int wave_max_i32(int x) {
  x = max(x, __builtin_amdgcn_mov_dpp(x, kDppQuadSwap1, 0xF, 0xF, false));
  x = max(x, __builtin_amdgcn_mov_dpp(x, kDppQuadSwap2, 0xF, 0xF, false));
  x = max(x, __builtin_amdgcn_mov_dpp(x, kDppHalfMirror, 0xF, 0xF, false));
  x = max(x, __builtin_amdgcn_mov_dpp(x, kDppMirror, 0xF, 0xF, false));
  return max(max(__builtin_amdgcn_readlane(x, 0), __builtin_amdgcn_readlane(x, 16)),
             max(__builtin_amdgcn_readlane(x, 32), __builtin_amdgcn_readlane(x, 48)));
}


// Camera constants, FP64, precomputed on the host.
struct CamConst {
  double eye[3], right[3], up[3], fwd[3];
  double th;      // tan(fov_y / 2), perspective
  double hw, hh;  // ortho_w / 2, ortho_h / 2, orthographic
  int32_t proj, W, H, pad;
};

struct VolConst {
  const void *data;
  int32_t dtype;
  int32_t nx, ny, nz;
  uint32_t bytes;           // total bytes (< 4 GiB)
  const float2 *minmax;     // per-block (min, max) or nullptr
  int32_t nbx, nby, nbz, edge;
  int32_t edge_shift;       // log2(edge)
  int32_t row_even;         // nx even: every x-row starts at an even element
  // per-launch block occupancy under the TF, bit b % 32 of word b / 32
  // (nullptr: decided from minmax and the TF on the fly)
  const uint32_t *occ = nullptr;
  // nonzero: after the occupancy bits, occ holds the 2-bit radius plane
  // (ceil(nb / 16) words; see empty_radius); leaps use cubes of empty blocks
  // up to this radius
  int32_t occ_radius = 0;
};

struct TfConst {
  const float *table;  // K x 4 fp32
  int32_t K;
  float v0, scale;     // u = (v - v0) * scale, scale = (K-1)/(v1-v0) in fp32
  uint32_t *status;    // device word set to 1 when the table holds an invalid node (nullptr: not reported)
};

struct MarchConst {
  float step;
  float ert;        // in (0,1) enables early termination
  int32_t skip;     // nonzero: skip samples in empty blocks
  // nonzero (kernels that visit every sample, with the blocks' min/max): a
  // sample in a block that is empty under the TF and constant over its
  // footprint takes that constant as its value, without reconstructing it
  // (every tap of its stencil holds it)
  int32_t flat;
};

// ---------------------------------------------------------------------------
// LDS state of a workgroup: the TF table and a prefix count of its non-zero
// extinction nodes (block occupancy in O(1)).  Carved out of dynamic LDS,
// sized by K.
// ---------------------------------------------------------------------------
typedef __attribute__((address_space(3))) uint32_t lds_u32;

struct TfShared {
  float4 *node;                // K nodes (r, g, b, sigma)
  int32_t *pref;               // K + 1: pref[j] = #{i < j : sigma_i != 0}
  unsigned long long *mask;    // ceil(K / 64) ballot words
  lds_u32 *occ;                // LDS copy of VolConst::occ when occ_lds
  bool occ_lds;
};

__host__ __device__ inline uint32_t tf_lds_bytes(int K) {
  uint32_t a = (uint32_t)K * 16u;
  uint32_t b = (((uint32_t)K + 1u) * 4u + 7u) & ~7u;
  uint32_t c = (((uint32_t)K + 63u) / 64u) * 8u;
  return a + b + c;
}

__device__ inline TfShared carve_tf(char *base, int K) {
  TfShared s;
  s.node = reinterpret_cast<float4 *>(base);
  s.pref = reinterpret_cast<int32_t *>(base + (uint32_t)K * 16u);
  s.mask = reinterpret_cast<unsigned long long *>(base + (uint32_t)K * 16u +
                                                  ((((uint32_t)K + 1u) * 4u + 7u) & ~7u));
  s.occ = nullptr;
  s.occ_lds = false;
  return s;
}

// A TF node is valid when all four channels are finite and the extinction is
// not negative.
__device__ inline bool tf_node_valid(float4 n) {
  return __builtin_isfinite(n.x) && __builtin_isfinite(n.y) && __builtin_isfinite(n.z) && __builtin_isfinite(n.w) &&
         n.w >= 0.0f;
}

__device__ inline float4 nan_rgba() {
  const float q = __builtin_nanf("");
  return make_float4(q, q, q, q);
}

// Load the TF into LDS and build the prefix counts.  All 256 threads call it.
// Returns false (uniformly) when some node is invalid: the caller then writes
// NaN results instead of rendering, the status word records it, and every
// block counts as occupied (negative or NaN extinction is read as zero in the
// LDS copy, so nothing downstream sees it).
template <int NT = kWgSize>  // threads of the workgroup
__device__ inline bool load_tf(TfShared &s, const TfConst &tf) {
  const int t = threadIdx.x;
  const float4 *src = reinterpret_cast<const float4 *>(tf.table);
  int bad = 0;
  for (int j = t; j < tf.K; j += NT) {
    float4 n = src[j];
    bad |= tf_node_valid(n) ? 0 : 1;
    n.w = fmaxf(n.w, 0.0f);
    s.node[j] = n;
  }
  bad = __syncthreads_or(bad);
  const int words = (tf.K + 63) / 64;
  const int wave = t / kWaveSize, lane = t % kWaveSize;
  for (int w = wave; w < words; w += NT / kWaveSize) {
    int j = w * 64 + lane;
    bool nz = (j < tf.K) && (bad || s.node[j].w != 0.0f);
    unsigned long long m = __ballot(nz);
    if (lane == 0) s.mask[w] = m;
  }
  __syncthreads();
  for (int j = t; j <= tf.K; j += NT) {
    int w = j / 64, b = j % 64;
    int c = 0;
    for (int q = 0; q < w; ++q) c += __popcll(s.mask[q]);
    if (w < words && b) c += __popcll(s.mask[w] & ((1ull << b) - 1ull));
    s.pref[j] = c;
  }
  __syncthreads();
  if (bad && t == 0 && tf.status) __hip_atomic_store(tf.status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return !bad;
}

// Occupancy of a block with value range [mn, mx]: some node in
// [floor(u(mn)) - 1, ceil(u(mx)) + 1] (clamped) has non-zero extinction.
__device__ inline bool range_occupied(const TfShared &s, int K, float v0, float scale, float mn, float mx) {
  float ulo = (mn - v0) * scale;
  float uhi = (mx - v0) * scale;
  ulo = fminf(fmaxf(ulo, -2.0f), (float)K + 1.0f);
  uhi = fminf(fmaxf(uhi, -2.0f), (float)K + 1.0f);
  int jlo = (int)floorf(ulo) - 1;
  int jhi = (int)ceilf(uhi) + 1;
  jlo = min(max(jlo, 0), K - 1);
  jhi = min(max(jhi, 0), K - 1);
  return s.pref[jhi + 1] - s.pref[jlo] > 0;
}

// ---------------------------------------------------------------------------
// Ray setup (FP64).  The expression order matches the camera definition in
// vr.h term by term and no operation is contracted into an FMA, so the
// lattice count -- an integer decided by floating point -- is reproducible.
// ---------------------------------------------------------------------------
struct Ray {
  float p0[3];  // entry point o + t_in d, rounded to fp32
  float d[3];   // unit direction, rounded to fp32
  float s0;     // t_{k0} - t_in, in (0, step]
  int32_t k0;   // first lattice index: smallest k with (k + 1/2) step > t_in
  int32_t ns;   // lattice samples: k0 <= k < k0 + ns
  bool hit;
};

// The ray moves from its origin with the fixed step; lattice samples sit at
// t_k = (k + 1/2) step, every k >= 0 with t_in < t_k < t_out.  Rays of
// neighbouring pixels share sample distances, so a wavefront's samples at one
// k lie on a thin slab.  Sample k is at p0 + (s0 + (k - k0) step) d.
__device__ inline Ray setup_ray(const CamConst &c, int col, int row, int nx, int ny, int nz, float step32) {
#pragma clang fp contract(off)
  Ray r;
  r.hit = false;
  r.ns = 0;
  r.k0 = 0;
  r.s0 = 0.0f;
  double sx = 2.0 * ((double)col + 0.5) / (double)c.W - 1.0;
  double sy = 1.0 - 2.0 * ((double)row + 0.5) / (double)c.H;
  double o[3], d[3];
  if (c.proj != 0) {
    double a = sx * c.th * ((double)c.W / (double)c.H);
    double b = sy * c.th;
    for (int k = 0; k < 3; ++k) {
      o[k] = c.eye[k];
      d[k] = c.fwd[k] + a * c.right[k] + b * c.up[k];
    }
  } else {
    double a = sx * c.hw;
    double b = sy * c.hh;
    for (int k = 0; k < 3; ++k) {
      o[k] = c.eye[k] + a * c.right[k] + b * c.up[k];
      d[k] = c.fwd[k];
    }
  }
  double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
  for (int k = 0; k < 3; ++k) d[k] = d[k] / n;
  // slab clip against [-1/2, n - 1/2]^3
  double hi[3] = {(double)nx - 0.5, (double)ny - 0.5, (double)nz - 0.5};
  double t0 = -INFINITY, t1 = INFINITY;
  for (int a = 0; a < 3; ++a) {
    if (d[a] == 0.0) {
      if (o[a] < -0.5 || o[a] > hi[a]) return r;
      continue;
    }
    double ta = (-0.5 - o[a]) / d[a];
    double tb = (hi[a] - o[a]) / d[a];
    if (ta > tb) {
      double s = ta;
      ta = tb;
      tb = s;
    }
    if (ta > t0) t0 = ta;
    if (tb < t1) t1 = tb;
  }
  double te = t0 > 0.0 ? t0 : 0.0;
  if (!(t1 > te)) return r;
  // lattice: smallest k >= 0 with (k + 1/2) step > te, then every k while
  // (k + 1/2) step < t1 (the predicates of the definition, in FP64)
  double st = (double)step32;
  double est = floor(te / st - 0.5);
  long long k = est > 0.0 ? (long long)est : 0;
  while (k > 0 && ((double)(k - 1) + 0.5) * st > te) --k;
  while (((double)k + 0.5) * st <= te) ++k;
  long long k0 = k;
  double est1 = ceil(t1 / st - 0.5);
  long long k1 = est1 > (double)k0 ? (long long)est1 : k0;
  while (k1 > k0 && ((double)(k1 - 1) + 0.5) * st >= t1) --k1;
  while (((double)k1 + 0.5) * st < t1) ++k1;
  r.k0 = (int32_t)k0;
  r.ns = (int32_t)(k1 - k0);
  r.hit = r.ns > 0;
  r.s0 = (float)(((double)k0 + 0.5) * st - te);
  for (int a = 0; a < 3; ++a) {
    r.p0[a] = (float)(o[a] + te * d[a]);
    r.d[a] = (float)d[a];
  }
  return r;
}

// ---------------------------------------------------------------------------
// Tricubic B-spline reconstruction.
// ---------------------------------------------------------------------------
__device__ inline void bspline_weights(float t, float w[4]) {
  const float s = 1.0f - t;
  const float t2 = t * t, t3 = t2 * t;
  w[0] = (1.0f / 6.0f) * s * s * s;
  w[3] = (1.0f / 6.0f) * t3;
  w[1] = fmaf(0.5f, t3, (2.0f / 3.0f) - t2);
  w[2] = 1.0f - w[0] - w[1] - w[3];
}

typedef uint32_t u32x3 __attribute__((ext_vector_type(3)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ inline __amdgpu_buffer_rsrc_t make_rsrc(const void *p, uint32_t bytes) {
  // raw buffer: stride 0, num_records in bytes; dword format word for gfx9
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, 0x00020000);
}

template <int DT> struct Vox;

template <> struct Vox<kI16> {
  static constexpr int kBytes = 2;
  // even-length rows: byte offset of the pair-aligned window `voff` (per
  // lane), row offset `soff` (uniform, in the SGPR soffset), shift `sh`;
  // row_s_load + row_unpack are the same in two parts (loads ahead of use)
  using RawRow = u32x3;
  __device__ static inline RawRow row_s_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b96(r, voff, soff, 0);
  }
  __device__ static inline void row_unpack(const RawRow &v, uint32_t sh, float t[4]) {
    uint32_t lo = __builtin_amdgcn_alignbit(v.y, v.x, sh);
    uint32_t hi = __builtin_amdgcn_alignbit(v.z, v.y, sh);
    t[0] = (float)(int16_t)(lo & 0xffffu);
    t[1] = (float)((int32_t)lo >> 16);
    t[2] = (float)(int16_t)(hi & 0xffffu);
    t[3] = (float)((int32_t)hi >> 16);
  }
  __device__ static inline void row_s(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, uint32_t sh,
                                      float t[4]) {
    u32x3 v = __builtin_amdgcn_raw_buffer_load_b96(r, voff, soff, 0);
    uint32_t lo = __builtin_amdgcn_alignbit(v.y, v.x, sh);
    uint32_t hi = __builtin_amdgcn_alignbit(v.z, v.y, sh);
    t[0] = (float)(int16_t)(lo & 0xffffu);
    t[1] = (float)((int32_t)lo >> 16);
    t[2] = (float)(int16_t)(hi & 0xffffu);
    t[3] = (float)((int32_t)hi >> 16);
  }
  // four consecutive taps starting at element e; e_al = e & ~1 even
  __device__ static inline void row(__amdgpu_buffer_rsrc_t r, uint32_t e, float t[4]) {
    uint32_t ea = e & ~1u;
    u32x3 v = __builtin_amdgcn_raw_buffer_load_b96(r, ea * 2u, 0, 0);
    uint32_t sh = (e & 1u) * 16u;
    uint32_t lo = __builtin_amdgcn_alignbit(v.y, v.x, sh);
    uint32_t hi = __builtin_amdgcn_alignbit(v.z, v.y, sh);
    t[0] = (float)(int16_t)(lo & 0xffffu);
    t[1] = (float)((int32_t)lo >> 16);
    t[2] = (float)(int16_t)(hi & 0xffffu);
    t[3] = (float)((int32_t)hi >> 16);
  }
  __device__ static inline float one(__amdgpu_buffer_rsrc_t r, uint32_t e) {
    return (float)(int16_t)__builtin_amdgcn_raw_buffer_load_b16(r, e * 2u, 0, 0);
  }
  // the dwordx3 window of the row starting at e lies inside the buffer
  __device__ static inline bool window_ok(uint32_t e, uint32_t nvox) { return (e & ~1u) + 6u <= nvox; }
  // 16 consecutive voxels from element e: the 9-dword window from e & ~1,
  // loaded by row16_load and converted by row16_unpack (so that a caller can
  // keep several rows in flight)
  __device__ static inline bool row16_ok(uint32_t e, uint32_t nvox) { return (e & ~1u) + 18u <= nvox; }
  struct Raw {
    u32x4 p, q;
    uint32_t z;
  };
  __device__ static inline Raw row16_load(__amdgpu_buffer_rsrc_t r, uint32_t e) {
    const uint32_t b = (e & ~1u) * 2u;
    return Raw{__builtin_amdgcn_raw_buffer_load_b128(r, b, 0, 0), __builtin_amdgcn_raw_buffer_load_b128(r, b + 16u, 0, 0),
               __builtin_amdgcn_raw_buffer_load_b32(r, b + 32u, 0, 0)};
  }
  __device__ static inline void row16_unpack(const Raw &w, uint32_t e, float t[16]) {
    const uint32_t sh = (e & 1u) * 16u;
    const uint32_t d[9] = {w.p.x, w.p.y, w.p.z, w.p.w, w.q.x, w.q.y, w.q.z, w.q.w, w.z};
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      uint32_t x = __builtin_amdgcn_alignbit(d[j + 1], d[j], sh);
      t[2 * j] = (float)(int16_t)(x & 0xffffu);
      t[2 * j + 1] = (float)((int32_t)x >> 16);
    }
  }
};

template <> struct Vox<kU16> {
  static constexpr int kBytes = 2;
  using RawRow = u32x3;
  __device__ static inline RawRow row_s_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b96(r, voff, soff, 0);
  }
  __device__ static inline void row_unpack(const RawRow &v, uint32_t sh, float t[4]) {
    uint32_t lo = __builtin_amdgcn_alignbit(v.y, v.x, sh);
    uint32_t hi = __builtin_amdgcn_alignbit(v.z, v.y, sh);
    t[0] = (float)(lo & 0xffffu);
    t[1] = (float)(lo >> 16);
    t[2] = (float)(hi & 0xffffu);
    t[3] = (float)(hi >> 16);
  }
  __device__ static inline void row_s(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, uint32_t sh,
                                      float t[4]) {
    u32x3 v = __builtin_amdgcn_raw_buffer_load_b96(r, voff, soff, 0);
    uint32_t lo = __builtin_amdgcn_alignbit(v.y, v.x, sh);
    uint32_t hi = __builtin_amdgcn_alignbit(v.z, v.y, sh);
    t[0] = (float)(lo & 0xffffu);
    t[1] = (float)(lo >> 16);
    t[2] = (float)(hi & 0xffffu);
    t[3] = (float)(hi >> 16);
  }
  __device__ static inline void row(__amdgpu_buffer_rsrc_t r, uint32_t e, float t[4]) {
    uint32_t ea = e & ~1u;
    u32x3 v = __builtin_amdgcn_raw_buffer_load_b96(r, ea * 2u, 0, 0);
    uint32_t sh = (e & 1u) * 16u;
    uint32_t lo = __builtin_amdgcn_alignbit(v.y, v.x, sh);
    uint32_t hi = __builtin_amdgcn_alignbit(v.z, v.y, sh);
    t[0] = (float)(lo & 0xffffu);
    t[1] = (float)(lo >> 16);
    t[2] = (float)(hi & 0xffffu);
    t[3] = (float)(hi >> 16);
  }
  __device__ static inline float one(__amdgpu_buffer_rsrc_t r, uint32_t e) {
    return (float)(uint16_t)__builtin_amdgcn_raw_buffer_load_b16(r, e * 2u, 0, 0);
  }
  __device__ static inline bool window_ok(uint32_t e, uint32_t nvox) { return (e & ~1u) + 6u <= nvox; }
  __device__ static inline bool row16_ok(uint32_t e, uint32_t nvox) { return (e & ~1u) + 18u <= nvox; }
  using Raw = Vox<kI16>::Raw;
  __device__ static inline Raw row16_load(__amdgpu_buffer_rsrc_t r, uint32_t e) { return Vox<kI16>::row16_load(r, e); }
  __device__ static inline void row16_unpack(const Raw &w, uint32_t e, float t[16]) {
    const uint32_t sh = (e & 1u) * 16u;
    const uint32_t d[9] = {w.p.x, w.p.y, w.p.z, w.p.w, w.q.x, w.q.y, w.q.z, w.q.w, w.z};
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      uint32_t x = __builtin_amdgcn_alignbit(d[j + 1], d[j], sh);
      t[2 * j] = (float)(x & 0xffffu);
      t[2 * j + 1] = (float)(x >> 16);
    }
  }
};

template <> struct Vox<kF32> {
  static constexpr int kBytes = 4;
  using RawRow = u32x4;
  __device__ static inline RawRow row_s_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
    return __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
  }
  __device__ static inline void row_unpack(const RawRow &w, uint32_t, float t[4]) {
    const f32x4 v = __builtin_bit_cast(f32x4, w);
    t[0] = v.x;
    t[1] = v.y;
    t[2] = v.z;
    t[3] = v.w;
  }
  __device__ static inline void row_s(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff, uint32_t,
                                      float t[4]) {
    f32x4 v = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0));
    t[0] = v.x;
    t[1] = v.y;
    t[2] = v.z;
    t[3] = v.w;
  }
  __device__ static inline void row(__amdgpu_buffer_rsrc_t r, uint32_t e, float t[4]) {
    f32x4 v = __builtin_bit_cast(f32x4, __builtin_amdgcn_raw_buffer_load_b128(r, e * 4u, 0, 0));
    t[0] = v.x;
    t[1] = v.y;
    t[2] = v.z;
    t[3] = v.w;
  }
  __device__ static inline float one(__amdgpu_buffer_rsrc_t r, uint32_t e) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, e * 4u, 0, 0));
  }
  __device__ static inline bool window_ok(uint32_t, uint32_t) { return true; }
  __device__ static inline bool row16_ok(uint32_t, uint32_t) { return true; }
  struct Raw {
    u32x4 a[4];
  };
  __device__ static inline Raw row16_load(__amdgpu_buffer_rsrc_t r, uint32_t e) {
    Raw w;
#pragma unroll
    for (int j = 0; j < 4; ++j) w.a[j] = __builtin_amdgcn_raw_buffer_load_b128(r, (e + 4u * j) * 4u, 0, 0);
    return w;
  }
  __device__ static inline void row16_unpack(const Raw &w, uint32_t, float t[16]) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const f32x4 v = __builtin_bit_cast(f32x4, w.a[j]);
      t[4 * j] = v.x;
      t[4 * j + 1] = v.y;
      t[4 * j + 2] = v.z;
      t[4 * j + 3] = v.w;
    }
  }
};

// Stencil geometry of one sample: cell, fractional offsets, weights.
struct Stencil {
  int ix, iy, iz;
  float wx[4], wy[4], wz[4];
};

__device__ inline Stencil make_stencil(float px, float py, float pz) {
  Stencil s;
  float fx = floorf(px), fy = floorf(py), fz = floorf(pz);
  s.ix = (int)fx;
  s.iy = (int)fy;
  s.iz = (int)fz;
  bspline_weights(px - fx, s.wx);
  bspline_weights(py - fy, s.wy);
  bspline_weights(pz - fz, s.wz);
  return s;
}

// Catmull-Rom weights of the same four taps (interpolating; two negative).
__device__ inline void catmull_rom_weights(float t, float w[4]) {
  const float t2 = t * t, t3 = t2 * t;
  w[0] = 0.5f * (2.0f * t2 - t3 - t);
  w[1] = 0.5f * fmaf(3.0f, t3, fmaf(-5.0f, t2, 2.0f));
  w[2] = 0.5f * fmaf(-3.0f, t3, fmaf(4.0f, t2, t));
  w[3] = 0.5f * (t3 - t2);
}

// Trilinear weights on the same four taps: the two nearest only.
__device__ inline void trilinear_weights(float t, float w[4]) {
  w[0] = 0.0f;
  w[1] = 1.0f - t;
  w[2] = t;
  w[3] = 0.0f;
}

// Stencil with the filter's weights: F = 0 cubic B-spline, 1 Catmull-Rom,
// 3 trilinear.
template <int F>
__device__ inline Stencil make_stencil_f(float px, float py, float pz) {
  if constexpr (F == 0) {
    return make_stencil(px, py, pz);
  } else {
    Stencil s;
    float fx = floorf(px), fy = floorf(py), fz = floorf(pz);
    s.ix = (int)fx;
    s.iy = (int)fy;
    s.iz = (int)fz;
    if constexpr (F == 3) {
      trilinear_weights(px - fx, s.wx);
      trilinear_weights(py - fy, s.wy);
      trilinear_weights(pz - fz, s.wz);
    } else {
      catmull_rom_weights(px - fx, s.wx);
      catmull_rom_weights(py - fy, s.wy);
      catmull_rom_weights(pz - fz, s.wz);
    }
    return s;
  }
}

// Visit the 16 x-rows of a stencil's taps, row(c, b, t) with t[a] =
// V[iz-1+c][iy-1+b][ix-1+a] under clamp-to-edge addressing, in the order
// c = 0..3, b = 0..3.  Interior stencils take the packed-row loads.
template <int DT, class Row>
__device__ inline void for_rows(__amdgpu_buffer_rsrc_t rs, const VolConst &v, const Stencil &s, Row &row) {
  const int nx = v.nx, ny = v.ny, nz = v.nz;
  const uint32_t nxy = (uint32_t)nx * (uint32_t)ny;
  const uint32_t nvox = nxy * (uint32_t)nz;
  bool inner = (s.ix >= 1) & (s.ix + 2 <= nx - 1) & (s.iy >= 1) & (s.iy + 2 <= ny - 1) & (s.iz >= 1) &
               (s.iz + 2 <= nz - 1);
  if (inner) {
    uint32_t e0 = ((uint32_t)(s.iz - 1) * (uint32_t)ny + (uint32_t)(s.iy - 1)) * (uint32_t)nx + (uint32_t)(s.ix - 1);
    inner = Vox<DT>::window_ok(e0 + 3u * nxy + 3u * (uint32_t)nx, nvox);
    if (inner && (DT == kF32 || v.row_even)) {
      // every row has e0's parity: one per-lane window offset, the row
      // offsets are uniform and travel in the load's SGPR soffset
      const uint32_t kb = (uint32_t)Vox<DT>::kBytes;
      const uint32_t voff = (DT == kF32) ? e0 * 4u : (e0 & ~1u) * 2u;
      const uint32_t sh = (e0 & 1u) * 16u;
      const uint32_t rs_x = (uint32_t)nx * kb, rs_xy = nxy * kb;
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          float t[4];
          Vox<DT>::row_s(rs, voff, (uint32_t)c * rs_xy + (uint32_t)b * rs_x, sh, t);
          row(c, b, t);
        }
      return;
    }
    if (inner) {
#pragma unroll
      for (int c = 0; c < 4; ++c)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          float t[4];
          Vox<DT>::row(rs, e0 + (uint32_t)c * nxy + (uint32_t)b * (uint32_t)nx, t);
          row(c, b, t);
        }
      return;
    }
  }
  int xs[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) xs[a] = min(max(s.ix - 1 + a, 0), nx - 1);
  for (int c = 0; c < 4; ++c) {
    uint32_t z = (uint32_t)min(max(s.iz - 1 + c, 0), nz - 1);
    for (int b = 0; b < 4; ++b) {
      uint32_t y = (uint32_t)min(max(s.iy - 1 + b, 0), ny - 1);
      uint32_t rowb = (z * (uint32_t)ny + y) * (uint32_t)nx;
      float t[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) t[a] = Vox<DT>::one(rs, rowb + (uint32_t)xs[a]);
      row(c, b, t);
    }
  }
}

// v = sum_c wz_c sum_b wy_b sum_a wx_a V[z_c][y_b][x_a], separable (16
// x-rows, 4 y-sums, 1 z-sum).  Every reconstruction path keeps this order, so
// a value does not depend on where its taps came from.
__device__ inline float row_sum(const float w[4], const float t[4]) {
  float r = w[0] * t[0];
  r = fmaf(w[1], t[1], r);
  r = fmaf(w[2], t[2], r);
  return fmaf(w[3], t[3], r);
}

struct ValueRows {
  const Stencil &s;
  float acc, accy;
  __device__ inline void operator()(int c, int b, const float t[4]) {
    if (b == 0) accy = 0.0f;
    accy = fmaf(s.wy[b], row_sum(s.wx, t), accy);
    if (b == 3) acc = fmaf(s.wz[c], accy, acc);
  }
};

template <int DT>
__device__ inline float reconstruct(__amdgpu_buffer_rsrc_t rs, const VolConst &v, const Stencil &s) {
  ValueRows f{s, 0.0f, 0.0f};
  for_rows<DT>(rs, v, s, f);
  return f.acc;
}

// The first kRows of the 16 x-rows of the stencil at cell (ix, iy, iz),
// loaded ahead of the sample that needs them (for_rows' interior fast path
// only; else empty); the rest are loaded when the sample is taken.  Holding
// all 16 across the adjoint's step spilled registers; with 8 the queued
// adjoint fits 256 without spills (C1 fwd + adjoint 10.0 -> 9.0 ms, C3 292
// -> 252 ms, with the queue).
template <int DT> struct TapPrefetch {
  static constexpr int kRows = 8;
  typename Vox<DT>::RawRow raw[kRows];
  int ix, iy, iz;  // ix == INT_MIN: empty
  uint32_t sh, voff;
};

template <int DT>
__device__ inline void prefetch_taps(TapPrefetch<DT> &p, __amdgpu_buffer_rsrc_t rs, const VolConst &v, int ix, int iy,
                                     int iz) {
  p.ix = INT_MIN;
  const int nx = v.nx, ny = v.ny, nz = v.nz;
  const uint32_t nxy = (uint32_t)nx * (uint32_t)ny;
  const bool inner = (ix >= 1) & (ix + 2 <= nx - 1) & (iy >= 1) & (iy + 2 <= ny - 1) & (iz >= 1) & (iz + 2 <= nz - 1);
  if (!inner || !(DT == kF32 || v.row_even)) return;
  const uint32_t e0 = ((uint32_t)(iz - 1) * (uint32_t)ny + (uint32_t)(iy - 1)) * (uint32_t)nx + (uint32_t)(ix - 1);
  if (!Vox<DT>::window_ok(e0 + 3u * nxy + 3u * (uint32_t)nx, nxy * (uint32_t)nz)) return;
  const uint32_t kb = (uint32_t)Vox<DT>::kBytes;
  const uint32_t voff = (DT == kF32) ? e0 * 4u : (e0 & ~1u) * 2u;
  const uint32_t rs_x = (uint32_t)nx * kb, rs_xy = nxy * kb;
#pragma unroll
  for (int i = 0; i < TapPrefetch<DT>::kRows; ++i)
    p.raw[i] = Vox<DT>::row_s_load(rs, voff, (uint32_t)(i / 4) * rs_xy + (uint32_t)(i % 4) * rs_x);
  p.voff = voff;
  p.sh = (e0 & 1u) * 16u;
  p.ix = ix;
  p.iy = iy;
  p.iz = iz;
}

// reconstruct() from the prefetched rows when they are this stencil's (the
// same taps in the same order: bit-identical), else from memory.
template <int DT>
__device__ inline float reconstruct_prefetched(const TapPrefetch<DT> &p, __amdgpu_buffer_rsrc_t rs, const VolConst &v,
                                               const Stencil &s) {
  if (p.ix != s.ix || p.iy != s.iy || p.iz != s.iz) return reconstruct<DT>(rs, v, s);
  constexpr int NP = TapPrefetch<DT>::kRows;
  // the rows not loaded ahead, issued before the prefetched ones are used
  typename Vox<DT>::RawRow late[16 - NP];
  const uint32_t kb = (uint32_t)Vox<DT>::kBytes;
  const uint32_t rs_x = (uint32_t)v.nx * kb, rs_xy = (uint32_t)v.nx * (uint32_t)v.ny * kb;
#pragma unroll
  for (int i = NP; i < 16; ++i)
    late[i - NP] = Vox<DT>::row_s_load(rs, p.voff, (uint32_t)(i / 4) * rs_xy + (uint32_t)(i % 4) * rs_x);
  ValueRows f{s, 0.0f, 0.0f};
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int i = 4 * c + b;
      float t[4];
      Vox<DT>::row_unpack(i < NP ? p.raw[i < NP ? i : 0] : late[i < NP ? 0 : i - NP], p.sh, t);
      f(c, b, t);
    }
  return f.acc;
}

__device__ inline float combine(const Stencil &s, const float t[4][4][4]) {
  float acc = 0.0f;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    float accy = 0.0f;
#pragma unroll
    for (int b = 0; b < 4; ++b) accy = fmaf(s.wy[b], row_sum(s.wx, t[c][b]), accy);
    acc = fmaf(s.wz[c], accy, acc);
  }
  return acc;
}

// The 64 taps as values: row visitor that stores each row.
struct TapRows {
  float (*t)[4][4];
  __device__ inline void operator()(int c, int b, const float r[4]) {
#pragma unroll
    for (int a = 0; a < 4; ++a) t[c][b][a] = r[a];
  }
};

template <int DT>
__device__ inline void load_taps(__amdgpu_buffer_rsrc_t rs, const VolConst &v, const Stencil &s, float t[4][4][4]) {
  TapRows f{t};
  for_rows<DT>(rs, v, s, f);
}

// Derivatives of the B-spline weights with respect to the offset t.
__device__ inline void bspline_dweights(float t, float d[4]) {
  const float s = 1.0f - t;
  d[0] = -0.5f * s * s;
  d[1] = t * fmaf(1.5f, t, -2.0f);
  d[2] = fmaf(t, fmaf(-1.5f, t, 1.0f), 0.5f);
  d[3] = 0.5f * t * t;
}

// A stencil with derivative weights: the gradient of the reconstructed field
// (the cubic filter's own gradient, used for local lighting).
struct StencilG {
  Stencil s;
  float dx[4], dy[4], dz[4];
};

__device__ inline StencilG make_stencil_grad(float px, float py, float pz) {
  StencilG g;
  g.s = make_stencil(px, py, pz);
  bspline_dweights(px - floorf(px), g.dx);
  bspline_dweights(py - floorf(py), g.dy);
  bspline_dweights(pz - floorf(pz), g.dz);
  return g;
}

// (value, dv/dx, dv/dy, dv/dz).  The value is combine()'s, bit for bit; each
// derivative swaps one axis' weights for derivative weights in the same
// separable order.
struct GradRows {
  const StencilG &g;
  float acc, ax, ay, az, accy, accx, accd;
  __device__ inline void operator()(int c, int b, const float t[4]) {
    if (b == 0) accy = accx = accd = 0.0f;
    const float r = row_sum(g.s.wx, t), rd = row_sum(g.dx, t);
    accy = fmaf(g.s.wy[b], r, accy);
    accx = fmaf(g.s.wy[b], rd, accx);
    accd = fmaf(g.dy[b], r, accd);
    if (b == 3) {
      acc = fmaf(g.s.wz[c], accy, acc);
      ax = fmaf(g.s.wz[c], accx, ax);
      ay = fmaf(g.s.wz[c], accd, ay);
      az = fmaf(g.dz[c], accy, az);
    }
  }
};

template <int DT>
__device__ inline float4 reconstruct_grad(__amdgpu_buffer_rsrc_t rs, const VolConst &v, const StencilG &g) {
  GradRows f{g, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  for_rows<DT>(rs, v, g.s, f);
  return make_float4(f.acc, f.ax, f.ay, f.az);
}

__device__ inline float4 combine_grad(const StencilG &g, const float t[4][4][4]) {
  GradRows f{g, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int c = 0; c < 4; ++c)
#pragma unroll
    for (int b = 0; b < 4; ++b) f(c, b, t[c][b]);
  return make_float4(f.acc, f.ax, f.ay, f.az);
}

// ---------------------------------------------------------------------------
// Value box: each wavefront stages in LDS a 14 x 14 x ZD (x, y, z) box of the
// volume over the slab its lanes are sampling, converted to fp32 with
// clamp-to-edge applied while filling.  ZD = 14, or 13 (kVBoxShallow): its
// 182 rows of 14 voxels fill in three passes of the wavefront's lanes where
// 196 need a fourth for 4 rows, while a deeper box is re-placed less often.
// The whole-image forward takes the shallow box for volumes the 256 MB MALL
// holds (C1 frame 1.233 -> 1.217 ms, C0 0.133 -> 0.122 ms) and the deep one
// for larger volumes, whose refills come from HBM (C2 frame 13.0 ms deep,
// 14.0 ms shallow).  Rows of 16 voxels or 12 rows per slice measured slower.  A step whose stencils all lie in the box reads its 64 taps
// per sample from LDS, with the same FMA order as the global path (the value
// is bit-identical).  When a step's stencils leave the box, the box is
// refilled around them, extended along the marching direction; a step whose
// stencils spread wider than the box reads from global memory.
// ---------------------------------------------------------------------------
#ifndef VR_VBOX_X
#define VR_VBOX_X 14
#endif
#ifndef VR_VBOX_Y
#define VR_VBOX_Y 14
#endif
#ifndef VR_VBOX_Z
#define VR_VBOX_Z 14
#endif
#ifndef VR_VBOX_ZPAD
#define VR_VBOX_ZPAD 2  // z stride 198 (C1 with ray pairs: 0 or 2 1.297 ms, 4 1.320, 6 1.61)
#endif
constexpr int kVBoxExt[3] = {VR_VBOX_X, VR_VBOX_Y, VR_VBOX_Z};  // extent per axis
constexpr int kVBox = VR_VBOX_X;                               // row stride (x)
constexpr int kVBoxRows = VR_VBOX_Y;                           // rows per slice (y)
constexpr int kVBoxZ = kVBox * kVBoxRows + VR_VBOX_ZPAD;       // padded z stride (LDS banks)
static_assert(VR_VBOX_ZPAD % 2 == 0, "slices hold float2 pairs");
static_assert(kVBox % 2 == 0 && kVBox >= 4 && kVBox <= 16, "box rows are filled in pairs from a 16-voxel window");
static_assert(VR_VBOX_Y >= 4 && VR_VBOX_Z >= 4, "a stencil fits the box");
constexpr int kVBoxCells = VR_VBOX_Z * kVBoxZ;
constexpr int kVBoxShallow = VR_VBOX_Z - 1;  // the shallow box's depth

struct ValBox {
  float *cells;  // this wavefront's LDS cells or nullptr (no staging)
  int ox, oy, oz;
  bool valid;
};

// kBatch rows per lane are loaded before any is stored (all of them by
// default; kernels short of registers take fewer).
template <int DT, int kBatch = (kVBoxRows * VR_VBOX_Z + kWaveSize - 1) / kWaveSize, int ZD = VR_VBOX_Z>
__device__ inline void vbox_fill(ValBox &b, __amdgpu_buffer_rsrc_t rs, const VolConst &v) {
  static_assert(ZD >= 4 && ZD <= VR_VBOX_Z, "the box's depth fits its cells");
  constexpr int kRows = kVBoxRows * ZD;
  constexpr int kPer = (kRows + kWaveSize - 1) / kWaveSize;  // rows per lane
  const int lane = threadIdx.x % kWaveSize;
  const uint32_t nvox = (uint32_t)v.nx * (uint32_t)v.ny * (uint32_t)v.nz;
  const bool x_in = b.ox >= 0 && b.ox + 15 <= v.nx - 1;
  auto batch = [&](int j0) {
    // first the 16-voxel windows of the batch's rows, so that their loads
    // are in flight together (every load is bounds-checked by the hardware,
    // so the windows of rows that take the clamped path below are harmless)
    uint32_t base[kBatch];
    typename Vox<DT>::Raw raw[kBatch];
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int row = min(lane + (j0 + j) * kWaveSize, kRows - 1);
      const uint32_t y = (uint32_t)min(max(b.oy + row % kVBoxRows, 0), v.ny - 1);
      const uint32_t z = (uint32_t)min(max(b.oz + row / kVBoxRows, 0), v.nz - 1);
      base[j] = (z * (uint32_t)v.ny + y) * (uint32_t)v.nx;
      raw[j] = Vox<DT>::row16_load(rs, base[j] + (uint32_t)max(b.ox, 0));
    }
#pragma unroll
    for (int j = 0; j < kBatch; ++j) {
      const int row = lane + (j0 + j) * kWaveSize;
      if (j0 + j < kPer && row < kRows) {
        const uint32_t rowbase = base[j];
        float t[16];  // a 16-voxel window; the first kVBox are stored
        if (x_in && Vox<DT>::row16_ok(rowbase + (uint32_t)b.ox, nvox)) {
          Vox<DT>::row16_unpack(raw[j], rowbase + (uint32_t)b.ox, t);
        } else {
#pragma unroll
          for (int i = 0; i < kVBox; ++i)
            t[i] = Vox<DT>::one(rs, rowbase + (uint32_t)min(max(b.ox + i, 0), v.nx - 1));
        }
        float2 *dst = reinterpret_cast<float2 *>(b.cells + (row / kVBoxRows) * kVBoxZ + (row % kVBoxRows) * kVBox);
#pragma unroll
        for (int i = 0; i < kVBox / 2; ++i) dst[i] = make_float2(t[2 * i], t[2 * i + 1]);
      }
    }
  };
  if constexpr (kBatch >= kPer) {
    batch(0);
  } else {
#pragma unroll 1
    for (int j0 = 0; j0 < kPer; j0 += kBatch) batch(j0);
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Wavefront-wide, before the samples of a step.
template <int DT, int kBatch = (kVBoxRows * VR_VBOX_Z + kWaveSize - 1) / kWaveSize, int ZD = VR_VBOX_Z>
__device__ inline void vbox_prepare(ValBox &b, __amdgpu_buffer_rsrc_t rs, const VolConst &v, const Ray &r,
                                    bool want, float px, float py, float pz) {
  int lo[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, hi[3] = {-0x7fffffff, -0x7fffffff, -0x7fffffff};
  if (want) {
    lo[0] = (int)floorf(px) - 1;
    lo[1] = (int)floorf(py) - 1;
    lo[2] = (int)floorf(pz) - 1;
#pragma unroll
    for (int a = 0; a < 3; ++a) hi[a] = lo[a] + 3;
  }
  const int o[3] = {b.ox, b.oy, b.oz};
  bool inside = true;
  if (want)
#pragma unroll
    for (int a = 0; a < 3; ++a) inside = inside && lo[a] >= o[a] && hi[a] < o[a] + (a == 2 ? ZD : kVBoxExt[a]);
  if (b.valid && __ballot(!inside) == 0ull) return;
  int mn[3], mx[3];
  bool fits = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    mn[a] = wave_min_i32(lo[a]);
    mx[a] = wave_max_i32(hi[a]);
    fits = fits && (mx[a] - mn[a] < (a == 2 ? ZD : kVBoxExt[a]));
  }
  if (!fits) {
    b.valid = false;  // this step reads from global memory
    return;
  }
  const unsigned long long wm = __ballot(want);
  const int first = __ffsll((long long)wm) - 1;
  int org[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float da = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, r.d[a]), first));
    org[a] = da >= 0.0f ? mn[a] : mx[a] - (a == 2 ? ZD : kVBoxExt[a]) + 1;
  }
  // the lanes may still read the previous contents: order the refill after them
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  b.ox = __builtin_amdgcn_readfirstlane(org[0]);
  b.oy = __builtin_amdgcn_readfirstlane(org[1]);
  b.oz = __builtin_amdgcn_readfirstlane(org[2]);
  vbox_fill<DT, kBatch, ZD>(b, rs, v);
  b.valid = true;
}

__device__ inline void load_taps_box(const ValBox &b, const Stencil &s, float t[4][4][4]) {
  const float *base = b.cells + (s.iz - 1 - b.oz) * kVBoxZ + (s.iy - 1 - b.oy) * kVBox + (s.ix - 1 - b.ox);
  // one base per z slice keeps the row offsets within the immediate offsets
  // of paired LDS reads
  typedef __attribute__((address_space(3))) const float lds_float;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    lds_float *zb = (lds_float *)(base + c * kVBoxZ);
    // keep each slice base in its own register (otherwise rows past the
    // 255-dword immediate range get one address add per LDS read)
    asm volatile("" : "+v"(zb));
#pragma unroll
    for (int bb = 0; bb < 4; ++bb)
#pragma unroll
      for (int a = 0; a < 4; ++a) t[c][bb][a] = zb[bb * kVBox + a];
  }
}

// All 64 taps from the box first, then the separable FMA chain of the
// global path (the value is bit-identical).
__device__ inline float reconstruct_box(const ValBox &b, const Stencil &s) {
  float t[4][4][4];
  load_taps_box(b, s, t);
  return combine(s, t);
}

// LDS bytes of the TF staging rounded up to 16, where the value boxes begin.
__host__ __device__ inline uint32_t vbox_lds_offset(int K) { return (tf_lds_bytes(K) + 15u) & ~15u; }
__host__ __device__ inline uint32_t vbox_lds_bytes() { return (uint32_t)(kWgSize / kWaveSize) * kVBoxCells * 4u; }

// ---------------------------------------------------------------------------
// Local lighting (Phong's model in the Blinn half-vector form, two-sided),
// with the gradient of the cubic reconstruction as the surface normal:
//   c' = c (ka + kd |n.L|) + ks |n.H|^shininess,
// n = -grad / max(|grad|, grad_min), V = -d, L = V for a headlight, H =
// (L + V) / |L + V| (0 when L = -V).  Opacity is not changed.
// ---------------------------------------------------------------------------
struct ShadeConst {
  float ka, kd, ks, shininess;
  float light[3];      // unit, towards the light (unused with a headlight)
  int32_t headlight;
  float grad_min;      // > 0
  int32_t pad;
};

struct RayLight {
  float L[3], H[3];
};

__device__ inline RayLight ray_light(const ShadeConst &sc, const float d[3]) {
  RayLight q;
  float h[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    q.L[a] = sc.headlight ? -d[a] : sc.light[a];
    h[a] = q.L[a] - d[a];
  }
  const float hn = sqrtf(fmaf(h[0], h[0], fmaf(h[1], h[1], h[2] * h[2])));
  const float inv = hn > 1e-12f ? 1.0f / hn : 0.0f;
#pragma unroll
  for (int a = 0; a < 3; ++a) q.H[a] = h[a] * inv;
  return q;
}

// Light colour c of a sample with gradient (g.y, g.z, g.w) (g.x is the value).
__device__ inline void light_colour(const ShadeConst &sc, const RayLight &q, const float4 &g, float4 &c) {
  const float gm = sqrtf(fmaf(g.y, g.y, fmaf(g.z, g.z, g.w * g.w)));
  const float inv = -1.0f / fmaxf(gm, sc.grad_min);
  const float n0 = g.y * inv, n1 = g.z * inv, n2 = g.w * inv;
  const float nl = fabsf(fmaf(n0, q.L[0], fmaf(n1, q.L[1], n2 * q.L[2])));
  const float nh = fabsf(fmaf(n0, q.H[0], fmaf(n1, q.H[1], n2 * q.H[2])));
  // nh^shininess through the hardware log2/exp2 (nh = 0 gives exp2(-inf) = 0)
  const float spec = sc.ks * __builtin_amdgcn_exp2f(sc.shininess * __builtin_amdgcn_logf(nh));
  const float f = fmaf(sc.kd, nl, sc.ka);
  c.x = fmaf(c.x, f, spec);
  c.y = fmaf(c.y, f, spec);
  c.z = fmaf(c.z, f, spec);
}

// Post-classification: (r, g, b, sigma) at value v; j and w of the segment;
// `clamped` when u fell outside [0, K-1].
struct Classified {
  float4 c;
  int j;
  float w;
  bool clamped;
};

__device__ inline Classified classify(const TfShared &s, int K, float v0, float scale, float v) {
  Classified q;
  float u = (v - v0) * scale;
  q.clamped = !(u >= 0.0f && u <= (float)(K - 1));
  u = fminf(fmaxf(u, 0.0f), (float)(K - 1));
  int j = min((int)u, K - 2);
  float w = u - (float)j;
  float4 a = s.node[j], b = s.node[j + 1];
  q.c.x = fmaf(w, b.x - a.x, a.x);
  q.c.y = fmaf(w, b.y - a.y, a.y);
  q.c.z = fmaf(w, b.z - a.z, a.z);
  q.c.w = fmaf(w, b.w - a.w, a.w);
  q.j = j;
  q.w = w;
  return q;
}

// Pre-classification: every tap classified, the opacity-weighted channels
// (sigma r, sigma g, sigma b, sigma) interpolated with the stencil's weights
// (separable, x rows then y then z); the colour is the weighted colour over
// the extinction, 0 where that is 0.
__device__ inline Classified preclassify(const TfShared &s, int K, float v0, float scale, const Stencil &st,
                                         const float t[4][4][4]) {
  float4 acc = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    float4 accy = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      float4 r = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const Classified q = classify(s, K, v0, scale, t[c][b][a]);
        const float ws = st.wx[a] * q.c.w;
        r.x = fmaf(ws, q.c.x, r.x);
        r.y = fmaf(ws, q.c.y, r.y);
        r.z = fmaf(ws, q.c.z, r.z);
        r.w = fmaf(st.wx[a], q.c.w, r.w);
      }
      accy.x = fmaf(st.wy[b], r.x, accy.x);
      accy.y = fmaf(st.wy[b], r.y, accy.y);
      accy.z = fmaf(st.wy[b], r.z, accy.z);
      accy.w = fmaf(st.wy[b], r.w, accy.w);
    }
    acc.x = fmaf(st.wz[c], accy.x, acc.x);
    acc.y = fmaf(st.wz[c], accy.y, acc.y);
    acc.z = fmaf(st.wz[c], accy.z, acc.z);
    acc.w = fmaf(st.wz[c], accy.w, acc.w);
  }
  Classified out;
  const float inv = acc.w > 0.0f ? 1.0f / acc.w : 0.0f;
  out.c = make_float4(acc.x * inv, acc.y * inv, acc.z * inv, acc.w);
  out.j = 0;
  out.w = 0.0f;
  out.clamped = false;
  return out;
}

// exp(-x) for x >= 0 via the hardware exp2 (1 ulp); x = sigma * step.
__device__ inline float transmit(float sigma, float step_log2e) {
  return __builtin_amdgcn_exp2f(-sigma * step_log2e);
}

// ---------------------------------------------------------------------------
// Empty-space leaping.  Block of the (clamped) cell of p, and the first
// lattice index that may leave it.
// ---------------------------------------------------------------------------
__device__ inline void block_coords(const VolConst &v, int ix, int iy, int iz, int bc[3]) {
  bc[0] = min(max(ix, 0), v.nx - 1) >> v.edge_shift;
  bc[1] = min(max(iy, 0), v.ny - 1) >> v.edge_shift;
  bc[2] = min(max(iz, 0), v.nz - 1) >> v.edge_shift;
}

__device__ inline int block_index(const VolConst &v, const int bc[3]) {
  return bc[0] + v.nbx * (bc[1] + v.nby * bc[2]);
}

__device__ inline int block_of_cell(const VolConst &v, int ix, int iy, int iz, int bc[3]) {
  block_coords(v, ix, iy, iz, bc);
  return block_index(v, bc);
}

__device__ inline int block_of(const VolConst &v, float px, float py, float pz, int bc[3]) {
  return block_of_cell(v, (int)floorf(px), (int)floorf(py), (int)floorf(pz), bc);
}

// 1 / x in FP64: the hardware reciprocal refined by two Newton steps (a few
// ulp of error, far inside the margins of leap_target).
__device__ inline double recip64(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// Every lattice index k' with k <= k' < result samples strictly inside the
// current block: positions fl(fma(s, d, p0)) are monotone in s per axis, and
// the bound is pulled in by 2^-9 voxel (more than the fp32 rounding of any
// position below 8192) and by one more full step.  Computed in FP64 (the
// quotients through recip64: errors of order 1e-16 relative).
//
// With rad > 0 every block within Chebyshev distance rad of the current one
// is empty too, and the bound is the exit from that cube of blocks (on a
// side where the cube reaches the edge of the grid the ray leaves the volume
// first).
__device__ inline int leap_target(const VolConst &v, const Ray &r, const int bc[3], float step, int k, int rad = 0) {
  const int nb[3] = {v.nbx, v.nby, v.nbz};
  double smin = INFINITY;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    double da = (double)r.d[a];
    double pa = (double)r.p0[a];
    if (da > 0.0 && bc[a] + rad < nb[a] - 1) {
      double bound = (double)((bc[a] + rad + 1) << v.edge_shift) - 0x1p-9;
      smin = fmin(smin, (bound - pa) * recip64(da));
    } else if (da < 0.0 && bc[a] - rad > 0) {
      double bound = (double)((bc[a] - rad) << v.edge_shift) + 0x1p-9;
      smin = fmin(smin, (bound - pa) * recip64(da));
    }
  }
  if (!(smin < 1e30)) return 0x7fffffff;
  // first j with s0 + j step >= smin, minus one step of margin
  double jf = ceil((smin - (double)r.s0) * recip64((double)step)) - 1.0;
  if (jf > 2.0e9) return 0x7fffffff;
  int kt = r.k0 + (int)fmax(jf, 0.0);
  return max(kt, k + 1);
}

// Position of lattice index k.
__device__ inline void lattice_point(const Ray &r, float step, int k, float &px, float &py, float &pz) {
  float sk = fmaf((float)(k - r.k0), step, r.s0);
  px = fmaf(sk, r.d[0], r.p0[0]);
  py = fmaf(sk, r.d[1], r.p0[1]);
  pz = fmaf(sk, r.d[2], r.p0[2]);
}

// Blocks' minmax and TF decide occupancy.
__device__ inline bool block_occupied(const VolConst &v, const TfShared &s, const TfConst &tf, int b);
__device__ inline int empty_radius(const VolConst &v, int b);

// Walk one ray's lattice with the whole wavefront in step: all lanes look at
// the same index k (a thin slab of the tile's rays).  A lane sits out when k
// is outside its ray, after its ray terminated, or when its sample lies in a
// block that is empty under the TF (such a sample would add exactly zero).
// When no lane has a sample to evaluate, the wavefront leaps to the smallest
// index any lane may need: its next lattice start, or the first index that
// may leave its empty block -- or the cube of empty blocks around it, when
// the launch carries the radius plane (the lane sits out until then, without
// looking at its samples).  prep(want, px, py, pz) runs on every lane of the
// wavefront before the samples of a step (for wavefront-wide staging);
// visit(k, px, py, pz) evaluates one sample and returns false to stop the ray.
// post() runs on every lane after the samples of a step.
struct NoPrep {
  __device__ inline void operator()(bool, float, float, float) const {}
};
struct NoPost {
  __device__ inline void operator()() const {}
};

// FROM: start at lattice index kstart (>= r.k0) instead of r.k0 -- a ray
// resumed where an earlier pass left it; positions still follow r.
template <class Visit, class Prep, class Post, bool FROM = false>
__device__ inline void walk(const VolConst &v, const TfShared &s, const TfConst &tf, const MarchConst &mc,
                            const Ray &r, Visit &visit, Prep &prep, Post &post, int kstart = 0) {
  const int kb = r.hit ? (FROM ? max(r.k0, kstart) : r.k0) : 0x7fffffff;
  const int ke = r.hit ? r.k0 + r.ns : 0;
  bool alive = r.hit;
  int k = wave_min_i32(kb);
  const int kend = wave_max_i32(ke);
  int kfree = kb;  // indices below kfree: before the ray, or left in an empty block
  // the grid constants of the per-step block lookup and leap held in
  // registers, so the loop does not re-read them from the kernel arguments
  // (a scalar load whose wait also drains the wavefront's LDS reads)
  VolConst vg = v;
  asm volatile("" : "+v"(vg.nx), "+v"(vg.ny), "+v"(vg.nz), "+v"(vg.edge_shift), "+v"(vg.nbx), "+v"(vg.nby));
  int cur_block = -1;
  bool cur_occ = false;
  int bc[3] = {0, 0, 0};
  while (k < kend) {
    const bool in = alive && k >= kfree && k < ke;
    bool want = in;
    // every lane computes its position and cell (used by in-lanes only), so the
    // floors dominate, and are shared with, the box test and the stencil
    float px, py, pz;
    lattice_point(r, mc.step, k, px, py, pz);
    const int ix = (int)floorf(px), iy = (int)floorf(py), iz = (int)floorf(pz);
    if (in && mc.skip) {
      const int b = block_of_cell(vg, ix, iy, iz, bc);
      if (b != cur_block) {
        cur_block = b;
        cur_occ = block_occupied(v, s, tf, b);
      }
      want = cur_occ;
    }
    if (__ballot(want) == 0ull) {
      if (in) kfree = leap_target(vg, r, bc, mc.step, k, empty_radius(v, cur_block));
      const int prop = alive && k < ke ? kfree : 0x7fffffff;
      const int m = wave_min_i32(prop);
      k = m > k + 1 ? m : k + 1;
      continue;
    }
    prep(want, px, py, pz);
    if (want && !visit(k, px, py, pz)) alive = false;
    post();
    ++k;
  }
}

// ---------------------------------------------------------------------------
// Ray groups.  G consecutive lanes (within a quad) march one ray: at each step
// of the wavefront, lane j of a group takes lattice index k + j and the
// wavefront advances G indices.  A wavefront then holds 64 / G rays and
// finishes them in about 1 / G of the steps, so the longest tiles of an image
// -- the rays through the whole volume, which set a kernel's length -- are
// split into G times as many, G times shorter pieces of work.
//
// Each lane evaluates its own sample (skipping, leaps and staging as in walk);
// the group's G samples are then composited front to back in index order by
// every lane of the group, with the one-lane march's operations in its order,
// so colour, transmittance and the termination sample are bit-identical to
// it.  A sample the ray does not take (outside its extent, in an empty block,
// or after the step's sample that ended it) enters the chain as the identity
// (c = 0, transmittance 1), which changes nothing exactly.
// ---------------------------------------------------------------------------

// Lane I of each ray group, to every lane of the group (a DPP quad
// permutation: [I, I, 2 + I, 2 + I] for pairs, [I, I, I, I] for quads).
template <int G, int I>
__device__ inline float from_group_lane(float x) {
  if constexpr (G == 1) {
    return x;
  } else {
    constexpr int hi = G == 2 ? 2 + I : I;
    constexpr int ctrl = I | (I << 2) | (hi << 4) | (hi << 6);
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, x), ctrl, 0xF, 0xF, false));
  }
}

// A classified sample as it enters the compositing chain: colour and
// transmittance exp(-sigma step).
struct ChainSample {
  float c0, c1, c2, e;
};

// The state of a ray after one of its samples: T_k a_k of that sample, and
// colour and transmittance after it.
struct ChainState {
  float ta, C0, C1, C2, T;
};

// walk for ray groups.  eval(k, px, py, pz) -> ChainSample evaluates this
// lane's sample (called only where the ray takes it); take(mine, own) runs on
// every lane after the chain, `mine` telling whether this lane's sample was
// composited and `own` the ray's state right after it; prep and post as in
// walk.  acc carries the ray's (C0, C1, C2, T) in and out.
//
// FLAT (kernels that visit every sample, mc.flat set): a sample in a block
// that is empty under the TF and constant over its footprint is not
// evaluated; its value is that constant and it changes neither colour nor
// transmittance, so the ray's samples in such a block form a run of identical
// samples in an unchanging state.  flat(n, own, value) accounts for n of them
// at once: each lane for its own sample of a step, and when no lane of the
// wavefront has a sample to evaluate the wavefront leaps (as over empty
// blocks) and the first lane of each group with a flat sample also accounts
// for the indices the leap passes over -- every one inside that lane's block
// (the leap ends at or before its block's exit) and not past the ray's end.
// Every lattice index is accounted exactly once.
struct NoFlat {
  __device__ inline void operator()(int, const ChainState &, float) const {}
};

//
// STOP: a sample whose eval returns a negative transmittance (kStopSample)
// stops its ray before it: it is not composited, nor is any later sample of
// its step, and walk_group returns its index (else -1) -- a pass that does
// not hold the sample's data parks the ray there.  kstart >= 0 resumes a ray
// at lattice index max(k0, kstart).
constexpr float kStopSample = -1.0f;

template <int G, bool FLAT = false, bool STOP = false, class Eval, class Prep, class Take, class Flat, class Post>
__device__ inline int walk_group(const VolConst &v, const TfShared &s, const TfConst &tf, const MarchConst &mc,
                                 const Ray &r, Eval &eval, Prep &prep, Take &take, Flat &flat, Post &post,
                                 float4 &acc, int kstart = -1) {
  const int lane = (int)(threadIdx.x % kWaveSize);
  const int j = lane % G;  // this lane's place in its group
  const bool ert_on = mc.ert > 0.0f && mc.ert < 1.0f;
  float C0 = acc.x, C1 = acc.y, C2 = acc.z, T = acc.w;
  int stopped = -1;
  const int kb = r.hit ? (kstart >= 0 ? max(r.k0, kstart) : r.k0) : 0x7fffffff;
  const int ke = r.hit ? r.k0 + r.ns : 0;
  bool alive = r.hit;
  int k = wave_min_i32(kb);
  const int kend = wave_max_i32(ke);
  int kfree = kb;  // indices below kfree: before the ray, or left in an empty block
  VolConst vg = v;
  asm volatile("" : "+v"(vg.nx), "+v"(vg.ny), "+v"(vg.nz), "+v"(vg.edge_shift), "+v"(vg.nbx), "+v"(vg.nby));
  int cur_block = -1;
  bool cur_occ = false, cur_flat = false;
  float cur_value = 0.0f;
  int bc[3] = {0, 0, 0};
  const bool flat_on = FLAT && mc.flat && !mc.skip;
  const bool by_block = mc.skip || flat_on;
  while (k < kend) {
    const int kk = k + j;
    const bool in = alive && kk >= kfree && kk < ke;
    bool want = in, is_flat = false;
    float px, py, pz;
    lattice_point(r, mc.step, kk, px, py, pz);
    const int ix = (int)floorf(px), iy = (int)floorf(py), iz = (int)floorf(pz);
    if (in && by_block) {
      // the adjoint's every-sample walk forms the block's index only when its
      // coordinates change (measured faster there; the skipping forward
      // compares indices)
      int b;
      bool changed;
      if constexpr (FLAT) {
        const int ox = bc[0], oy = bc[1], oz = bc[2];
        block_coords(vg, ix, iy, iz, bc);
        changed = cur_block < 0 || bc[0] != ox || bc[1] != oy || bc[2] != oz;
        b = changed ? block_index(vg, bc) : cur_block;
      } else {
        b = block_of_cell(vg, ix, iy, iz, bc);
        changed = b != cur_block;
      }
      if (changed) {
        cur_block = b;
        cur_occ = block_occupied(v, s, tf, b);
        if constexpr (FLAT) {
          const float2 mm = v.minmax[b];
          cur_flat = flat_on && !cur_occ && mm.x == mm.y;
          cur_value = mm.x;
        }
      }
      if (mc.skip) want = cur_occ;
      if constexpr (FLAT) {
        is_flat = cur_flat;
        want = want && !is_flat;
      }
    }
    if (__ballot(want) == 0ull) {
      // no lane takes a sample at k .. k + G - 1: leap to the smallest index
      // any lane may need (every index below it is known to be unneeded or,
      // flat, accounted below)
      int prop = alive && kk < ke ? kfree : 0x7fffffff;
      if (in) {
        const int t = leap_target(vg, r, bc, mc.step, kk, empty_radius(v, cur_block));
        if (is_flat)
          prop = t;  // (a flat run is accounted, never skipped: kfree stays)
        else
          prop = kfree = t;
      }
      const int m = wave_min_i32(prop);
      const int knext = m > k + G ? m : k + G;
      if constexpr (FLAT) {
        const unsigned long long fm = __ballot(is_flat);
        if (is_flat) {
          const unsigned gb = (unsigned)(fm >> (lane - j)) & ((1u << G) - 1u);
          const bool first = (gb & ((1u << j) - 1u)) == 0u;
          const int n = 1 + (first ? max(min(knext, ke) - (k + G), 0) : 0);
          flat(n, ChainState{0.0f, C0, C1, C2, T}, cur_value);
        }
      }
      k = knext;
      continue;
    }
    prep(want, px, py, pz);
    ChainSample q = {0.0f, 0.0f, 0.0f, 1.0f};  // the identity unless taken
    if (want) q = eval(kk, px, py, pz);
    bool live = alive, mine = false, mine_flat = false;
    ChainState own = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    auto link = [&](auto I_) {
      constexpr int I = decltype(I_)::value;
      const float ei = from_group_lane<G, I>(q.e), xi = from_group_lane<G, I>(q.c0);
      const float yi = from_group_lane<G, I>(q.c1), zi = from_group_lane<G, I>(q.c2);
      const bool at = j == I;
      if constexpr (STOP) {
        if (ei < 0.0f && live) {  // kStopSample: the ray stops before this sample
          stopped = k + I;
          live = false;
        }
      }
      if (at) {
        mine = want && live;
        mine_flat = is_flat && live;
      }
      const float ee = live ? ei : 1.0f;
      const float ta = T * (1.0f - ee);
      C0 = fmaf(ta, xi, C0);
      C1 = fmaf(ta, yi, C1);
      C2 = fmaf(ta, zi, C2);
      T = T * ee;
      if (at) own = ChainState{ta, C0, C1, C2, T};
      if (ert_on && (1.0f - T) >= mc.ert) live = false;
    };
    link(std::integral_constant<int, 0>{});
    if constexpr (G > 1) link(std::integral_constant<int, 1>{});
    if constexpr (G > 2) {
      link(std::integral_constant<int, 2>{});
      link(std::integral_constant<int, 3>{});
    }
    alive = live;
    take(mine, own);
    if constexpr (FLAT)
      if (mine_flat) flat(1, own, cur_value);
    post();
    k += G;
  }
  acc = make_float4(C0, C1, C2, T);
  return stopped;
}

__device__ inline bool block_occupied(const VolConst &v, const TfShared &s, const TfConst &tf, int b) {
  if (s.occ_lds) return (s.occ[b >> 5] >> (b & 31)) & 1u;
  if (v.occ) return (v.occ[b >> 5] >> (b & 31)) & 1u;
  float2 mm = v.minmax[b];
  return range_occupied(s, tf.K, tf.v0, tf.scale, mm.x, mm.y);
}

// Chebyshev radius (in blocks, at most kEmptyRadiusMax) around the empty
// block b within which every block is empty: the 2-bit radius plane after the
// occupancy bits, when the launch has it (else 0).
__device__ inline int empty_radius(const VolConst &v, int b) {
  if (!v.occ || !v.occ_radius) return 0;
  const int64_t words = ((int64_t)v.nbx * v.nby * v.nbz + 31) / 32;
  return min((int)(v.occ[words + (b >> 4)] >> (2 * (b & 15))) & 3, v.occ_radius);
}

// Copy the occupancy bits of a launch into LDS at `dst` (all threads of the
// workgroup; visible after the next barrier).
__device__ inline void stage_occupancy(TfShared &s, const VolConst &v, char *dst, int words) {
  s.occ = (lds_u32 *)dst;
  s.occ_lds = true;
  for (int j = threadIdx.x; j < words; j += kWgSize) s.occ[j] = v.occ[j];
}

// ---------------------------------------------------------------------------
// Tile mapping.  A workgroup owns a 16x16 super-tile; wavefront w the 8x8
// sub-tile (w & 1, w >> 1); lane l the pixel (l & 7, l >> 3) of it.
// Super-tiles are grouped in chunks of ce x ce (ce = 4: 64x64 pixels).  The
// hardware hands workgroup i to XCD i mod 8; workgroup i works on chunk
// g = 8 (i / 8 / ce^2) + (i mod 8), so XCD x runs the chunks g = x (mod 8) one
// after another and the workgroups of a chunk share that XCD's L2.  Chunks
// are numbered along a Morton curve (over the chunk grid padded to a power of
// two), so the chunks of one XCD are spread evenly over the image and every
// XCD gets a similar share of the dense centre.
// ---------------------------------------------------------------------------
struct SuperTile {
  int view, sx, sy;  // super-tile coordinates within the view
  bool valid;
};

__host__ __device__ inline int pow2_at_least(int n) {
  int p = 1;
  while (p < n) p <<= 1;
  return p;
}

__host__ __device__ inline int64_t grid_size_for(int W, int H, int views, int ce) {
  int stx = (W + kSuperEdge - 1) / kSuperEdge, sty = (H + kSuperEdge - 1) / kSuperEdge;
  int cx = (stx + ce - 1) / ce, cy = (sty + ce - 1) / ce;
  int p = pow2_at_least(cx > cy ? cx : cy);
  int64_t nc = (int64_t)p * p * views;
  int64_t per = (int64_t)ce * ce;
  return ((nc + kXcds - 1) / kXcds) * kXcds * per;
}

__host__ __device__ inline int compact_bits(uint32_t m) {
  m &= 0x55555555u;
  m = (m | (m >> 1)) & 0x33333333u;
  m = (m | (m >> 2)) & 0x0f0f0f0fu;
  m = (m | (m >> 4)) & 0x00ff00ffu;
  m = (m | (m >> 8)) & 0x0000ffffu;
  return (int)m;
}

__device__ inline SuperTile map_workgroup(int64_t wg, int W, int H, int views, int ce) {
  SuperTile st;
  const int per = ce * ce;
  const int64_t xcd = wg % kXcds, r = wg / kXcds;
  const int64_t g = (r / per) * kXcds + xcd;
  const int pos = (int)(r % per);
  const int stx = (W + kSuperEdge - 1) / kSuperEdge, sty = (H + kSuperEdge - 1) / kSuperEdge;
  const int cx = (stx + ce - 1) / ce, cy = (sty + ce - 1) / ce;
  const int p = pow2_at_least(cx > cy ? cx : cy);
  const int64_t per_view = (int64_t)p * p;
  st.view = (int)(g / per_view);
  const uint32_t m = (uint32_t)(g % per_view);
  const int ccx = compact_bits(m), ccy = compact_bits(m >> 1);
  st.sx = ccx * ce + pos % ce;
  st.sy = ccy * ce + pos / ce;
  st.valid = st.view < views && ccx < cx && ccy < cy && st.sx < stx && st.sy < sty;
  return st;
}

// Workgroup -> super-tile through a precomputed order (item q = view * tiles
// + sy * tiles_x + sx), or the Morton chunk mapping when there is none.
__device__ inline SuperTile tile_of(const int32_t *order, int64_t wg, int W, int H, int views, int ce) {
  if (!order) return map_workgroup(wg, W, H, views, ce);
  const int tx = (W + kSuperEdge - 1) / kSuperEdge, ty = (H + kSuperEdge - 1) / kSuperEdge;
  const int q = order[wg], per = tx * ty;
  SuperTile st;
  st.view = q / per;
  st.sx = (q % per) % tx;
  st.sy = (q % per) / tx;
  st.valid = true;
  return st;
}

__device__ inline void pixel_of(int sx, int sy, int &col, int &row) {
  int wave = threadIdx.x / kWaveSize, lane = threadIdx.x % kWaveSize;
  col = sx * kSuperEdge + (wave & 1) * kTileEdge + (lane & 7);
  row = sy * kSuperEdge + (wave >> 1) * kTileEdge + (lane >> 3);
}

// Workgroup -> (super-tile, part): with ray groups of G lanes a workgroup
// covers 16 / G rows of a 16x16 super-tile.  The G parts of super-tile item q
// are workgroups 8 G (q / 8) + 8 p + q % 8 (p < G), all on the XCD of q.
template <int G>
__device__ inline SuperTile group_tile_of(const int32_t *order, int64_t wg, int W, int H, int views, int ce,
                                          int &part) {
  const int64_t q = (wg / (kXcds * G)) * kXcds + wg % kXcds;
  part = (int)((wg / kXcds) % G);
  if (order && q >= (int64_t)views * ((W + kSuperEdge - 1) / kSuperEdge) * ((H + kSuperEdge - 1) / kSuperEdge)) {
    SuperTile st;
    st.view = st.sx = st.sy = 0;
    st.valid = false;
    return st;
  }
  return tile_of(order, q, W, H, views, ce);
}

// Pixel of the ray of thread t of a workgroup item: wavefront w = t / 64 of
// part p covers a TW x TH block (8x8, 8x4, 4x4 for G = 1, 2, 4), ray
// r = (t mod 64) / G the pixel (r mod TW, r / TW) of it.
template <int G>
__device__ inline void group_pixel_of(int sx, int sy, int part, int t, int &col, int &row) {
  constexpr int TW = G <= 2 ? 8 : 4, TH = kWaveSize / G / TW, WX = kSuperEdge / TW;
  const int wave = t / kWaveSize, ray = (t % kWaveSize) / G;
  col = sx * kSuperEdge + (wave % WX) * TW + ray % TW;
  row = sy * kSuperEdge + part * (kSuperEdge / G) + (wave / WX) * TH + ray / TW;
}

template <int G>
__device__ inline void group_pixel_of(int sx, int sy, int part, int &col, int &row) {
  group_pixel_of<G>(sx, sy, part, (int)threadIdx.x, col, row);
}

// Workgroups of a launch over `items` super-tile items (or the padded Morton
// grid) with ray groups of G lanes.
__host__ __device__ inline int64_t group_grid(int64_t items, int G) {
  return (items + kXcds - 1) / kXcds * kXcds * G;
}

// ---------------------------------------------------------------------------
// Wavefront work queues.  Within an XCD the hardware hands workgroups to its
// shader engines in strict rotation, and waits for the next one in turn to
// have room: when the long tiles pile up on one shader engine, the others
// idle although work is left (measured on the C1 frame: 15-40 % of some
// engines' slots idle in the middle of the launch).  A queued launch instead
// starts only as many workgroups as the device holds at once; each of their
// wavefronts takes wavefront items (wavefront w of workgroup item i) from a
// counter per XCD until its queue is drained.  Workgroup item i belongs to
// queue i mod 8 (the XCD it would have run on), queue position
// 4 (i / 8) + w; workgroup j's wavefronts drain queue j mod 8 only (so every
// queue is drained whatever XCD its workgroups land on, as long as the launch
// has at least eight; helping the other queues once their own is empty
// measured 2 % slower on the C1 frame).  The counters sit behind the
// workgroup order, in the same buffer, and are zeroed by the kernel that
// writes the order.
// ---------------------------------------------------------------------------
constexpr int kQueueStride = 32;                         // ints: one 128-byte line per counter
constexpr int64_t kOrderQueueInts = kXcds * kQueueStride;  // counters behind the order
constexpr int kWavesPerWg = kWgSize / kWaveSize;

// Take the next wavefront item (workgroup item i, wavefront w) of queue x;
// false once it is drained.  Called by the whole wavefront.
__device__ inline bool next_wave_item(uint32_t *queue, uint32_t per_queue, int x, int64_t &i, int &w) {
  uint32_t idx = 0;
  if (threadIdx.x % kWaveSize == 0) idx = atomicAdd(queue + x * kQueueStride, 1u);
  idx = __builtin_amdgcn_readfirstlane(idx);
  if (idx >= per_queue) return false;
  i = x + (int64_t)kXcds * (idx / kWavesPerWg);
  w = (int)(idx % kWavesPerWg);
  return true;
}

// The kernel's by-value argument struct, read in place from the kernarg
// segment (scalar loads; dynamic indexing then needs no private copy).
template <class T> __device__ inline const T &kernarg() {
  return *(const T *)__builtin_amdgcn_kernarg_segment_ptr();
}

// Diagnostics (a library built with VR_TIMELINE): lane 0 of a wavefront
// writes the record of its wavefront item w (start, end, super-tile << 32 |
// HW_ID, work) into `tl` (item w = 4 x workgroup item + wavefront).
constexpr int kTimelineWaves = 1 << 17;
#ifdef VR_TIMELINE
__device__ inline void timeline_record(unsigned long long *tl, size_t w, unsigned long long t0, int tile, uint32_t work) {
  for (int off = 32; off > 0; off >>= 1) work += __shfl_xor(work, off, kWaveSize);
  const unsigned long long t1 = __builtin_amdgcn_s_memrealtime();
  if (threadIdx.x % kWaveSize == 0 && w < (size_t)kTimelineWaves) {
    unsigned hw;
    asm volatile("s_getreg_b32 %0, hwreg(HW_REG_HW_ID)" : "=s"(hw));
    tl[w * 4 + 0] = t0;
    tl[w * 4 + 1] = t1;
    tl[w * 4 + 2] = ((unsigned long long)(unsigned)tile << 32) | hw;
    tl[w * 4 + 3] = work;
  }
}
#endif

// Sum a per-lane count over the wavefront and add it to a 64-bit counter.
__device__ inline void wave_count(unsigned long long *ctr, uint32_t v) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWaveSize);
  if ((threadIdx.x % kWaveSize) == 0 && v) atomicAdd(ctr, (unsigned long long)v);
}

}  // namespace vr
