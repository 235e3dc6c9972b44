// render_fwd.hip -- forward ray casting kernel (gfx950).
//
// Per pixel (Section 2 of the paper): cast a ray from the camera, clip it to
// the volume box, march the midpoint lattice with the fixed step, reconstruct
// the scalar with the tricubic B-spline, classify through the TF
// (post-classification), composite front to back, stop once the opacity
// reaches the threshold, and leap over blocks that cannot be visible.
#include <algorithm>

#include "vr_internal.h"

namespace vr {

// One sample's classified colour and extinction at (px, py, pz): the value (or,
// lit, value and gradient) reconstructed from the LDS box when the step's
// stencils lie in it, else from global memory, then classified through the TF
// (post-classification; pre-classification for F == 2).  SHADE lights the
// classified colour with the gradient of the same 64 taps (the value, hence
// opacity and termination, is unchanged).
template <int DT, bool SHADE, int F>
__device__ inline Classified eval_sample(const VolConst &v, const TfShared &s, const TfConst &tf, float tf_v0,
                                         float tf_scale, const ShadeConst &sc, const RayLight &rl,
                                         __amdgpu_buffer_rsrc_t rs, const ValBox &box, float px, float py, float pz,
                                         uint32_t &unstaged) {
  Classified q;
  if constexpr (SHADE) {
    StencilG sg = make_stencil_grad(px, py, pz);
    float4 vg;
    if (box.valid) {
      float t[4][4][4];
      load_taps_box(box, sg.s, t);
      vg = combine_grad(sg, t);
    } else {
      vg = reconstruct_grad<DT>(rs, v, sg);
      ++unstaged;
    }
    q = classify(s, tf.K, tf.v0, tf.scale, vg.x);
    light_colour(sc, rl, vg, q.c);
  } else if constexpr (F == 2) {
    Stencil st = make_stencil(px, py, pz);
    float t[4][4][4];
    if (box.valid) {
      load_taps_box(box, st, t);
    } else {
      load_taps<DT>(rs, v, st, t);
      ++unstaged;
    }
    q = preclassify(s, tf.K, tf.v0, tf.scale, st, t);
  } else {
    Stencil st = make_stencil_f<F>(px, py, pz);
    float val;
    if (box.valid) {
      val = reconstruct_box(box, st);
    } else {
      val = reconstruct<DT>(rs, v, st);
      ++unstaged;
    }
    q = classify(s, tf.K, tf_v0, tf_scale, val);
  }
  return q;
}

// March one ray front to back, one ray per lane.  Skipped samples are exactly
// those whose block is empty under the TF; such a sample would contribute
// a = 0 exactly, so the result is bit-identical to marching every sample.
template <int DT, bool SHADE, int F = 0>
__device__ inline float4 march(const VolConst &v, const TfShared &s, const TfConst &tf, const MarchConst &mc,
                               const ShadeConst &sc, const Ray &r, __amdgpu_buffer_rsrc_t rs, ValBox &box,
                               uint32_t &evaluated, uint32_t &unstaged) {
  float C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, T = 1.0f;
  const float sl2 = mc.step * 1.4426950408889634f;
  float tf_v0 = tf.v0, tf_scale = tf.scale;  // held in registers (as the walk's grid constants)
  asm volatile("" : "+v"(tf_v0), "+v"(tf_scale));
  const bool ert_on = mc.ert > 0.0f && mc.ert < 1.0f;
  RayLight rl;
  if constexpr (SHADE) rl = ray_light(sc, r.d);
  // lighting and pre-classification hold more registers: two box rows in
  // flight per lane
  constexpr int kFillBatch = SHADE || F == 2 ? 2 : 4;
  auto prep = [&](bool want, float px, float py, float pz) {
    if (box.cells) vbox_prepare<DT, kFillBatch>(box, rs, v, r, want, px, py, pz);
  };
  auto visit = [&](int, float px, float py, float pz) -> bool {
    const Classified q = eval_sample<DT, SHADE, F>(v, s, tf, tf_v0, tf_scale, sc, rl, rs, box, px, py, pz, unstaged);
    float e = transmit(q.c.w, sl2);
    float ta = T * (1.0f - e);
    C0 = fmaf(ta, q.c.x, C0);
    C1 = fmaf(ta, q.c.y, C1);
    C2 = fmaf(ta, q.c.z, C2);
    T = T * e;
    ++evaluated;
    return !(ert_on && (1.0f - T) >= mc.ert);
  };
  NoPost post;
  walk(v, s, tf, mc, r, visit, prep, post);
  return make_float4(C0, C1, C2, 1.0f - T);
}

// The whole-image kernel marches each ray with a group of kRayGroup lanes
// (see walk_group): pairs, measured against one and four lanes per ray.
#ifndef VR_RAY_GROUP
#define VR_RAY_GROUP 2
#endif
constexpr int kRayGroup = VR_RAY_GROUP;
static_assert(kRayGroup == 1 || kRayGroup == 2 || kRayGroup == 4, "ray groups lie within a quad");

template <int G, int DT, bool SHADE, int F, int ZD = VR_VBOX_Z>
__device__ inline float4 march_group(const VolConst &v, const TfShared &s, const TfConst &tf, const MarchConst &mc,
                                     const ShadeConst &sc, const Ray &r, __amdgpu_buffer_rsrc_t rs, ValBox &box,
                                     uint32_t &evaluated, uint32_t &unstaged) {
  const float sl2 = mc.step * 1.4426950408889634f;
  float tf_v0 = tf.v0, tf_scale = tf.scale;
  asm volatile("" : "+v"(tf_v0), "+v"(tf_scale));
  RayLight rl;
  if constexpr (SHADE) rl = ray_light(sc, r.d);
  constexpr int kFillBatch = SHADE || F == 2 ? 2 : 4;
  auto prep = [&](bool want, float px, float py, float pz) {
    if (box.cells) vbox_prepare<DT, kFillBatch, ZD>(box, rs, v, r, want, px, py, pz);
  };
  auto eval = [&](int, float px, float py, float pz) -> ChainSample {
    const Classified q = eval_sample<DT, SHADE, F>(v, s, tf, tf_v0, tf_scale, sc, rl, rs, box, px, py, pz, unstaged);
    return ChainSample{q.c.x, q.c.y, q.c.z, transmit(q.c.w, sl2)};
  };
  auto take = [&](bool mine, const ChainState &) { evaluated += mine ? 1u : 0u; };
  NoFlat flat;
  NoPost post;
  float4 acc = make_float4(0.0f, 0.0f, 0.0f, 1.0f);
  walk_group<G>(v, s, tf, mc, r, eval, prep, take, flat, post, acc);
  return make_float4(acc.x, acc.y, acc.z, 1.0f - acc.w);
}

// The LDS value boxes bound the workgroups per CU (14^3 boxes: three, i.e.
// three wavefronts per SIMD); the register budget is set to match.
#ifndef VR_FWD_MAX_WAVES
#define VR_FWD_MAX_WAVES 3
#endif
// Unlit 16-bit volumes: registers budgeted for three wavefronts per SIMD (C1:
// leaving the compiler free measured 1 % slower); fp32 volumes keep the free
// budget (the C3 forward measured 2 % slower with the limit).
#ifndef VR_FWD_MIN_WAVES
#define VR_FWD_MIN_WAVES 3
#endif
constexpr uint32_t kLdsPerCu = 160u * 1024u;  // gfx950
constexpr uint64_t kMallBytes = 256ull << 20;   // MI355X: 256 MB of Infinity Cache (MALL)
constexpr uint32_t kFwdWgPerCu = VR_FWD_MAX_WAVES;  // four wavefronts per workgroup, one per SIMD

// The occupancy bits join the LDS state (after the boxes) when three
// workgroups still fit on a compute unit; else the kernels read them from
// global memory.
int32_t occupancy_lds_words(const RenderArgs &a, uint32_t lds) {
  if (!a.use_box || !a.vol.occ) return 0;
  const int64_t words = ((int64_t)a.vol.nbx * a.vol.nby * a.vol.nbz + 31) / 32;
  return (int64_t)lds + words * 4 <= (int64_t)(kLdsPerCu / kFwdWgPerCu) ? (int32_t)words : 0;
}
#ifdef VR_TIMELINE
__device__ unsigned long long g_timeline_fwd[kTimelineWaves * 4];
static int64_t g_timeline_fwd_records = 0;
#endif

// One wavefront item: wavefront w of workgroup item i (a part of a
// super-tile); the counts of its samples are added to the caller's.
template <int DT, bool SHADE, int F, int ZD>
__device__ inline void render_wave_item(const RenderArgs &a, const TfShared &s, bool tf_ok, ValBox &box,
                                        __amdgpu_buffer_rsrc_t rs, int64_t i, int w, uint32_t &evaluated,
                                        uint32_t &unstaged, uint32_t &lattice, uint32_t &hits) {
#ifdef VR_TIMELINE
  const unsigned long long tl0 = __builtin_amdgcn_s_memrealtime();
#endif
  int part;
  const SuperTile st = group_tile_of<kRayGroup>(a.order, i, a.W, a.H, a.n_views, a.chunk_edge, part);
  if (!st.valid) return;  // uniform over the wavefront
  int col, row;
  group_pixel_of<kRayGroup>(st.sx, st.sy, part, w * kWaveSize + (int)(threadIdx.x % kWaveSize), col, row);
  const bool inside = col < a.W && row < a.H;
  const bool lead = (threadIdx.x % kRayGroup) == 0;  // the lane that stores its group's pixel
  if (!tf_ok) {  // uniform: an invalid TF gives NaN pixels
    if (inside && lead) reinterpret_cast<float4 *>(a.out)[((size_t)st.view * a.H + row) * a.W + col] = nan_rgba();
    return;
  }
  const CamConst &cam = a.cams[st.view];
  // every lane enters the march (it steps the wavefront in unison); pixels
  // outside the image carry an empty ray
  Ray r;
  r.hit = false;
  r.ns = 0;
  r.k0 = 0;
  if (inside) r = setup_ray(cam, col, row, a.vol.nx, a.vol.ny, a.vol.nz, a.mc.step);
#ifdef VR_TIMELINE
  const uint32_t before = evaluated;
#endif
  float4 rgba;
  if constexpr (kRayGroup == 1)
    rgba = march<DT, SHADE, F>(a.vol, s, a.tf, a.mc, a.shade, r, rs, box, evaluated, unstaged);
  else
    rgba = march_group<kRayGroup, DT, SHADE, F, ZD>(a.vol, s, a.tf, a.mc, a.shade, r, rs, box, evaluated, unstaged);
  if (inside && lead) {
    float4 *o = reinterpret_cast<float4 *>(a.out);
    o[((size_t)st.view * a.H + row) * a.W + col] = rgba;
  }
  lattice += lead ? (uint32_t)r.ns : 0u;
  hits += lead && r.hit ? 1u : 0u;
#ifdef VR_TIMELINE
  const int tx = (a.W + kSuperEdge - 1) / kSuperEdge, ty = (a.H + kSuperEdge - 1) / kSuperEdge;
  timeline_record(g_timeline_fwd, (size_t)i * kWavesPerWg + w, tl0, st.view * tx * ty + st.sy * tx + st.sx,
                  evaluated - before);
#endif
}

// ZD: depth of the LDS value boxes (see ValBox).
template <int DT, bool SHADE, int F, int ZD = VR_VBOX_Z>
__global__ __launch_bounds__(kWgSize) __attribute__((amdgpu_waves_per_eu(SHADE ? VR_FWD_MAX_WAVES : (DT == kF32 ? 1 : VR_FWD_MIN_WAVES), VR_FWD_MAX_WAVES)))
void k_render(const RenderArgs args) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const RenderArgs &a = kernarg<RenderArgs>();
  if (!a.queue) {  // one workgroup item per workgroup
    int part;
    if (!group_tile_of<kRayGroup>(a.order, blockIdx.x, a.W, a.H, a.n_views, a.chunk_edge, part).valid)
      return;  // uniform over the workgroup
  }
  TfShared s = carve_tf(lds, a.tf.K);
  if (a.occ_lds_words > 0)
    stage_occupancy(s, a.vol, lds + vbox_lds_offset(a.tf.K) + vbox_lds_bytes(), a.occ_lds_words);
  const bool tf_ok = load_tf(s, a.tf);
  __amdgpu_buffer_rsrc_t rs = make_rsrc(a.vol.data, a.vol.bytes);
  // the wavefront's LDS value box (its contents stay valid from one item to
  // the next: the volume is the launch's)
  ValBox box;
  box.valid = false;
  box.ox = box.oy = box.oz = 0;
  box.cells = a.use_box ? reinterpret_cast<float *>(lds + vbox_lds_offset(a.tf.K)) +
                              (threadIdx.x / kWaveSize) * kVBoxCells
                        : nullptr;
  uint32_t evaluated = 0, unstaged = 0, lattice = 0, hits = 0;
  if (!a.queue) {
    render_wave_item<DT, SHADE, F, ZD>(a, s, tf_ok, box, rs, blockIdx.x, (int)(threadIdx.x / kWaveSize), evaluated,
                                   unstaged, lattice, hits);
  } else {
    const int x = (int)(blockIdx.x % kXcds);
    int w = 0;
    int64_t i = 0;
    while (next_wave_item(a.queue, (uint32_t)a.queue_items, x, i, w))
      render_wave_item<DT, SHADE, F, ZD>(a, s, tf_ok, box, rs, i, w, evaluated, unstaged, lattice, hits);
  }
  if (a.counters) {
    wave_count(a.counters + 0, evaluated);
    wave_count(a.counters + 1, lattice);
    wave_count(a.counters + 2, hits);
    wave_count(a.counters + 3, unstaged);
  }
}

// Workgroups of `fn` the current device holds at once with `lds` bytes of
// LDS each (0 when it cannot be found out).
int64_t resident_workgroups(const void *fn, uint32_t lds) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, kWgSize, lds) != hipSuccess) {
    (void)hipGetLastError();
    return 0;
  }
  return (int64_t)cus * per;
}

template <bool SHADE, int F, int ZD = VR_VBOX_Z>
static hipError_t launch_render_as(const RenderArgs &a0, int64_t grid, uint32_t lds, hipStream_t s) {
  RenderArgs a = a0;
  const void *fn = a.vol.dtype == kU16   ? reinterpret_cast<const void *>(&k_render<kU16, SHADE, F, ZD>)
                   : a.vol.dtype == kI16 ? reinterpret_cast<const void *>(&k_render<kI16, SHADE, F, ZD>)
                                         : reinterpret_cast<const void *>(&k_render<kF32, SHADE, F, ZD>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  // with an order (and its queue counters) the launch is queued: as many
  // workgroups as the device holds, fed wavefront items
  a.queue = nullptr;
  a.queue_items = 0;
  if (a.order) {
    const int64_t resident = resident_workgroups(fn, lds);
    if (resident >= kXcds && resident < grid) {
      a.queue = reinterpret_cast<uint32_t *>(const_cast<int32_t *>(a.order) + tile_order_count(a));
      a.queue_items = (int32_t)(grid / kXcds * kWavesPerWg);
      grid = resident;
    }
  }
  switch (a.vol.dtype) {
  case kU16: hipLaunchKernelGGL((k_render<kU16, SHADE, F, ZD>), dim3((unsigned)grid), dim3(kWgSize), lds, s, a); break;
  case kI16: hipLaunchKernelGGL((k_render<kI16, SHADE, F, ZD>), dim3((unsigned)grid), dim3(kWgSize), lds, s, a); break;
  default: hipLaunchKernelGGL((k_render<kF32, SHADE, F, ZD>), dim3((unsigned)grid), dim3(kWgSize), lds, s, a); break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Centre-out workgroup order: a counting sort of the super-tiles by their
// distance to the projected volume centre (half-tile rings) and, within a
// ring, by angle around the centre (32 sectors), in one workgroup.  Item i of
// the order runs on XCD i mod 8, so the angular order spreads every XCD's
// tiles around each ring: an XCD does not inherit one side of the volume (in
// raster order the two sides of a ring alternate, and the XCDs of one parity
// took one side: 7.5 % more work on four of them for the C1 frame).  Items of
// one (ring, sector) key come in any order; the image does not depend on the
// order.
// ---------------------------------------------------------------------------
constexpr int kOrderRings = 256;
constexpr int kOrderSectors = 32;
constexpr int kOrderKeys = kOrderRings * kOrderSectors;
constexpr int kOrderThreads = 1024;
constexpr int kKeysPerThread = kOrderKeys / kOrderThreads;

struct OrderArgs {
  float cx[kMaxCamsPerLaunch], cy[kMaxCamsPerLaunch];  // centre, in super-tile units
  int32_t tx, ty, n_views;
};

__device__ inline int order_key(const OrderArgs &o, int q) {
  const int per = o.tx * o.ty, v = q / per, t = q % per;
  const float dx = (float)(t % o.tx) - o.cx[v], dy = (float)(t / o.tx) - o.cy[v];
  const float d = sqrtf(fmaf(dx, dx, dy * dy)) * 2.0f;
  const int ring = d < (float)(kOrderRings - 1) ? (int)d : kOrderRings - 1;
  const float turn = atan2f(dy, dx) * 0.15915494309189535f + 0.5f;  // in [0, 1]
  const int sector = min(max((int)(turn * (float)kOrderSectors), 0), kOrderSectors - 1);
  return ring * kOrderSectors + sector;
}

__global__ __launch_bounds__(kOrderThreads) void k_tile_order(const OrderArgs o, int32_t *order) {
  __shared__ int cnt[kOrderKeys];
  const int n = o.n_views * o.tx * o.ty;
  for (int i = threadIdx.x; i < kOrderKeys; i += kOrderThreads) cnt[i] = 0;
  for (int i = threadIdx.x; i < (int)kOrderQueueInts; i += kOrderThreads) order[n + i] = 0;  // queue counters
  __syncthreads();
  for (int q = threadIdx.x; q < n; q += kOrderThreads) atomicAdd(&cnt[order_key(o, q)], 1);
  __syncthreads();
  // exclusive prefix sum of the counts: each thread sums its run of keys, an
  // inclusive scan of those sums inside each wavefront, then the wavefront totals
  __shared__ int wsum[kOrderThreads / kWaveSize];
  const int lane = threadIdx.x % kWaveSize, wave = threadIdx.x / kWaveSize;
  int run[kKeysPerThread], c = 0;
#pragma unroll
  for (int i = 0; i < kKeysPerThread; ++i) {
    run[i] = cnt[threadIdx.x * kKeysPerThread + i];
    c += run[i];
  }
  int x = c;
#pragma unroll
  for (int off = 1; off < kWaveSize; off <<= 1) {
    const int y = __shfl_up(x, off, kWaveSize);
    if (lane >= off) x += y;
  }
  if (lane == kWaveSize - 1) wsum[wave] = x;
  __syncthreads();
  int before = x - c;
  for (int w = 0; w < wave; ++w) before += wsum[w];
#pragma unroll
  for (int i = 0; i < kKeysPerThread; ++i) {
    cnt[threadIdx.x * kKeysPerThread + i] = before;
    before += run[i];
  }
  __syncthreads();
  for (int q = threadIdx.x; q < n; q += kOrderThreads) order[atomicAdd(&cnt[order_key(o, q)], 1)] = q;
}

int64_t render_grid(const RenderArgs &a) {
  if (a.order)
    return (int64_t)a.n_views * ((a.W + kSuperEdge - 1) / kSuperEdge) * ((a.H + kSuperEdge - 1) / kSuperEdge);
  return grid_size_for(a.W, a.H, a.n_views, a.chunk_edge);
}

hipError_t launch_tile_order(const RenderArgs &a, int32_t *order, hipStream_t s) {
  OrderArgs o;
  o.tx = (a.W + kSuperEdge - 1) / kSuperEdge;
  o.ty = (a.H + kSuperEdge - 1) / kSuperEdge;
  o.n_views = a.n_views;
  const double p[3] = {0.5 * (a.vol.nx - 1), 0.5 * (a.vol.ny - 1), 0.5 * (a.vol.nz - 1)};
  for (int v = 0; v < a.n_views; ++v) {
    const CamConst &c = a.cams[v];
    double d[3], z = 0.0, x = 0.0, y = 0.0;
    for (int k = 0; k < 3; ++k) d[k] = p[k] - c.eye[k];
    for (int k = 0; k < 3; ++k) {
      z += d[k] * c.fwd[k];
      x += d[k] * c.right[k];
      y += d[k] * c.up[k];
    }
    double sx = 0.0, sy = 0.0;  // image centre when the volume centre does not project
    if (c.proj != 0) {
      if (z > 0.0) {
        sx = x / (z * c.th * ((double)c.W / (double)c.H));
        sy = y / (z * c.th);
      }
    } else {
      sx = c.hw > 0.0 ? x / c.hw : 0.0;
      sy = c.hh > 0.0 ? y / c.hh : 0.0;
    }
    const double col = (sx + 1.0) * 0.5 * c.W - 0.5, row = (1.0 - sy) * 0.5 * c.H - 0.5;
    o.cx[v] = (float)fmin(fmax((col + 0.5) / kSuperEdge - 0.5, -1e6), 1e6);
    o.cy[v] = (float)fmin(fmax((row + 0.5) / kSuperEdge - 0.5, -1e6), 1e6);
  }
  hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(kOrderThreads), 0, s, o, order);
  return hipGetLastError();
}

int64_t tile_order_count(const RenderArgs &a) {
  return (int64_t)a.n_views * ((a.W + kSuperEdge - 1) / kSuperEdge) * ((a.H + kSuperEdge - 1) / kSuperEdge);
}

int32_t *make_tile_order(const RenderArgs &a, hipStream_t s) {
  int32_t *order = nullptr;
  if (hipMallocAsync((void **)&order, (size_t)(tile_order_count(a) + kOrderQueueInts) * sizeof(int32_t), s) != hipSuccess)
    return nullptr;
  if (launch_tile_order(a, order, s) != hipSuccess) {
    (void)hipFreeAsync(order, s);
    return nullptr;
  }
  return order;
}

hipError_t launch_render(const RenderArgs &a0, hipStream_t s) {
  RenderArgs a = a0;
  const int64_t grid = group_grid(render_grid(a), kRayGroup);
  uint32_t lds = tf_lds_bytes(a.tf.K);
  const uint32_t with_box = vbox_lds_offset(a.tf.K) + vbox_lds_bytes();
  a.use_box = with_box <= max_lds_per_workgroup() ? 1 : 0;
  if (a.use_box) lds = with_box;
  a.occ_lds_words = occupancy_lds_words(a, lds);
  lds += (uint32_t)a.occ_lds_words * 4u;
  if (a.vol.dtype != kU16 && a.vol.dtype != kI16 && a.vol.dtype != kF32) return hipErrorInvalidValue;
#ifdef VR_TIMELINE
  g_timeline_fwd_records = grid * (kWgSize / kWaveSize);
#endif
  if (a.shaded) return launch_render_as<true, 0>(a, grid, lds, s);
  if (a.filter == 1) return launch_render_as<false, 1>(a, grid, lds, s);
  if (a.filter == 2) return launch_render_as<false, 2>(a, grid, lds, s);
  if (a.filter == 3) return launch_render_as<false, 3>(a, grid, lds, s);
  // the shallow value box for volumes the MALL holds (their refills are
  // cheap, its fill passes fewer), the deep one above
  if (a.use_box && a.vol.bytes <= kMallBytes) return launch_render_as<false, 0, kVBoxShallow>(a, grid, lds, s);
  return launch_render_as<false, 0>(a, grid, lds, s);
}

// Serving: kRayGroup workgroups per work item, a 16x16 super-tile of one
// admitted request, its rays marched by lane groups as in the whole-image
// kernel; the items of a launch may come from many requests of different
// volumes, sizes and TFs.  The per-ray arithmetic is the whole-image
// kernel's, so a request's pixels do not depend on what it is batched with.
__global__ __launch_bounds__(kWgSize) void k_serve(const ServeSlot *slots, const ServeItem *items, int lds_k,
                                                   int use_box, unsigned long long *samples) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const ServeItem it = items[blockIdx.x / kRayGroup];  // (the item's parts are consecutive workgroups)
  const int part = (int)(blockIdx.x % kRayGroup);
  const ServeSlot &sl = slots[it.slot];
  TfShared s = carve_tf(lds, sl.tf.K);
  const bool tf_ok = load_tf(s, sl.tf);
  int col, row;
  group_pixel_of<kRayGroup>(it.sx, it.sy, part, col, row);
  const bool inside = col < sl.cam.W && row < sl.cam.H;
  const bool lead = (threadIdx.x % kRayGroup) == 0;
  if (!tf_ok) {  // (the server validates every table at submit)
    if (inside && lead) reinterpret_cast<float4 *>(sl.out)[(size_t)row * sl.cam.W + col] = nan_rgba();
    return;
  }
  Ray r;
  r.hit = false;
  r.ns = 0;
  r.k0 = 0;
  if (inside) r = setup_ray(sl.cam, col, row, sl.vol.nx, sl.vol.ny, sl.vol.nz, sl.mc.step);
  __amdgpu_buffer_rsrc_t rs = make_rsrc(sl.vol.data, sl.vol.bytes);
  uint32_t evaluated = 0, unstaged = 0;
  ValBox box;
  box.valid = false;
  box.ox = box.oy = box.oz = 0;
  box.cells = use_box ? reinterpret_cast<float *>(lds + vbox_lds_offset(lds_k)) + (threadIdx.x / kWaveSize) * kVBoxCells
                      : nullptr;
  float4 rgba;
  const ShadeConst sc{};
  switch (sl.vol.dtype) {  // uniform over the workgroup
  case kU16: rgba = march_group<kRayGroup, kU16, false, 0>(sl.vol, s, sl.tf, sl.mc, sc, r, rs, box, evaluated, unstaged); break;
  case kI16: rgba = march_group<kRayGroup, kI16, false, 0>(sl.vol, s, sl.tf, sl.mc, sc, r, rs, box, evaluated, unstaged); break;
  default: rgba = march_group<kRayGroup, kF32, false, 0>(sl.vol, s, sl.tf, sl.mc, sc, r, rs, box, evaluated, unstaged); break;
  }
  if (inside && lead) reinterpret_cast<float4 *>(sl.out)[(size_t)row * sl.cam.W + col] = rgba;
  wave_count(samples, evaluated);
}

hipError_t launch_serve_batch(const ServeSlot *slots_dev, const ServeItem *items_dev, int32_t n_items,
                              int32_t max_tf_k, unsigned long long *samples, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  uint32_t lds = tf_lds_bytes(max_tf_k);
  const uint32_t with_box = vbox_lds_offset(max_tf_k) + vbox_lds_bytes();
  const int use_box = with_box <= max_lds_per_workgroup() ? 1 : 0;
  if (use_box) lds = with_box;
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&k_serve),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_serve, dim3((unsigned)(n_items * kRayGroup)), dim3(kWgSize), lds, s, slots_dev, items_dev,
                     max_tf_k, use_box, samples);
  return hipGetLastError();
}

#ifdef VR_TIMELINE
int64_t timeline_copy_fwd(unsigned long long *host, int64_t max) {
  const int64_t n = std::min<int64_t>(std::min<int64_t>(g_timeline_fwd_records, kTimelineWaves), max);
  if (hipDeviceSynchronize() != hipSuccess) return -1;
  if (n > 0 && hipMemcpyFromSymbol(host, HIP_SYMBOL(g_timeline_fwd), (size_t)n * 4 * sizeof(unsigned long long)) != hipSuccess)
    return -1;
  return g_timeline_fwd_records;
}
#endif

}  // namespace vr
