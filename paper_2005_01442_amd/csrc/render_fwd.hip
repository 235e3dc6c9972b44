// render_fwd.hip -- forward ray casting kernel (gfx950).
//
// Per pixel (Section 2 of the paper): cast a ray from the camera, clip it to
// the volume box, march the midpoint lattice with the fixed step, reconstruct
// the scalar with the tricubic B-spline, classify through the TF
// (post-classification), composite front to back, stop once the opacity
// reaches the threshold, and leap over blocks that cannot be visible.
#include "vr_internal.h"

namespace vr {

// March one ray.  Skipped samples are exactly the samples whose block is
// empty under the TF; such a sample would contribute a = 0 exactly, so the
// result is bit-identical to marching every sample.
template <int DT>
__device__ inline float4 march(const VolConst &v, const TfShared &s, const TfConst &tf, const MarchConst &mc,
                               const Ray &r, __amdgpu_buffer_rsrc_t rs, uint32_t &evaluated) {
  float C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, T = 1.0f;
  const float sl2 = mc.step * 1.4426950408889634f;
  const bool ert_on = mc.ert > 0.0f && mc.ert < 1.0f;
  const int ns = r.hit ? r.ns : 0;
  int k = 0;
  int cur_block = -1;  // last block looked up and whether it is occupied
  bool cur_occ = false;
  while (k < ns) {
    float sk = ((float)k + 0.5f) * mc.step;
    float px = fmaf(sk, r.d[0], r.p0[0]);
    float py = fmaf(sk, r.d[1], r.p0[1]);
    float pz = fmaf(sk, r.d[2], r.p0[2]);
    if (mc.skip) {
      int bc[3];
      int b = block_of(v, px, py, pz, bc);
      if (b != cur_block) {
        cur_block = b;
        cur_occ = block_occupied(v, s, tf, b);
      }
      while (!cur_occ) {
        k = leap_target(v, r, bc, mc.step, k);
        if (k >= ns) break;
        sk = ((float)k + 0.5f) * mc.step;
        px = fmaf(sk, r.d[0], r.p0[0]);
        py = fmaf(sk, r.d[1], r.p0[1]);
        pz = fmaf(sk, r.d[2], r.p0[2]);
        b = block_of(v, px, py, pz, bc);
        if (b != cur_block) {
          cur_block = b;
          cur_occ = block_occupied(v, s, tf, b);
        }
      }
      if (k >= ns) break;
    }
    Stencil st = make_stencil(px, py, pz);
    float val = reconstruct<DT>(rs, v, st);
    Classified q = classify(s, tf.K, tf.v0, tf.scale, val);
    float e = transmit(q.c.w, sl2);
    float ta = T * (1.0f - e);
    C0 = fmaf(ta, q.c.x, C0);
    C1 = fmaf(ta, q.c.y, C1);
    C2 = fmaf(ta, q.c.z, C2);
    T = T * e;
    ++evaluated;
    ++k;
    if (ert_on && (1.0f - T) >= mc.ert) break;
  }
  return make_float4(C0, C1, C2, 1.0f - T);
}

template <int DT>
__global__ __launch_bounds__(kWgSize) void k_render(const RenderArgs args) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const RenderArgs &a = kernarg<RenderArgs>();
  SuperTile st = map_workgroup(blockIdx.x, a.W, a.H, a.n_views, a.chunk_edge);
  if (!st.valid) return;  // uniform over the workgroup
  TfShared s = carve_tf(lds, a.tf.K);
  load_tf(s, a.tf);
  int col, row;
  pixel_of(st.sx, st.sy, col, row);
  const bool inside = col < a.W && row < a.H;
  const CamConst &cam = a.cams[st.view];
  uint32_t evaluated = 0, lattice = 0, hit = 0;
  float4 rgba = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
  if (inside) {
    Ray r = setup_ray(cam, col, row, a.vol.nx, a.vol.ny, a.vol.nz, a.mc.step);
    if (r.hit) {
      __amdgpu_buffer_rsrc_t rs = make_rsrc(a.vol.data, a.vol.bytes);
      rgba = march<DT>(a.vol, s, a.tf, a.mc, r, rs, evaluated);
      lattice = (uint32_t)r.ns;
      hit = r.ns > 0 ? 1u : 0u;
    }
    float4 *o = reinterpret_cast<float4 *>(a.out);
    o[((size_t)st.view * a.H + row) * a.W + col] = rgba;
  }
  if (a.counters) {
    wave_count(a.counters + 0, evaluated);
    wave_count(a.counters + 1, lattice);
    wave_count(a.counters + 2, hit);
  }
}

hipError_t launch_render(const RenderArgs &a, hipStream_t s) {
  int64_t grid = grid_size_for(a.W, a.H, a.n_views, a.chunk_edge);
  uint32_t lds = tf_lds_bytes(a.tf.K);
  switch (a.vol.dtype) {
  case kU16: hipLaunchKernelGGL(k_render<kU16>, dim3((unsigned)grid), dim3(kWgSize), lds, s, a); break;
  case kI16: hipLaunchKernelGGL(k_render<kI16>, dim3((unsigned)grid), dim3(kWgSize), lds, s, a); break;
  case kF32: hipLaunchKernelGGL(k_render<kF32>, dim3((unsigned)grid), dim3(kWgSize), lds, s, a); break;
  default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// Serving: one workgroup per work item, a 16x16 super-tile of one admitted
// request; the items of a launch may come from many requests of different
// volumes, sizes and TFs.  The per-ray arithmetic is the whole-image
// kernel's, so a request's pixels do not depend on what it is batched with.
__global__ __launch_bounds__(kWgSize) void k_serve(const ServeSlot *slots, const ServeItem *items) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const ServeItem it = items[blockIdx.x];
  const ServeSlot &sl = slots[it.slot];
  TfShared s = carve_tf(lds, sl.tf.K);
  load_tf(s, sl.tf);
  int col, row;
  pixel_of(it.sx, it.sy, col, row);
  if (col < sl.cam.W && row < sl.cam.H) {
    float4 rgba = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    Ray r = setup_ray(sl.cam, col, row, sl.vol.nx, sl.vol.ny, sl.vol.nz, sl.mc.step);
    if (r.hit) {
      __amdgpu_buffer_rsrc_t rs = make_rsrc(sl.vol.data, sl.vol.bytes);
      uint32_t evaluated = 0;
      switch (sl.vol.dtype) {
      case kU16: rgba = march<kU16>(sl.vol, s, sl.tf, sl.mc, r, rs, evaluated); break;
      case kI16: rgba = march<kI16>(sl.vol, s, sl.tf, sl.mc, r, rs, evaluated); break;
      default: rgba = march<kF32>(sl.vol, s, sl.tf, sl.mc, r, rs, evaluated); break;
      }
    }
    reinterpret_cast<float4 *>(sl.out)[(size_t)row * sl.cam.W + col] = rgba;
  }
}

hipError_t launch_serve_batch(const ServeSlot *slots_dev, const ServeItem *items_dev, int32_t n_items,
                              int32_t max_tf_k, hipStream_t s) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_serve, dim3((unsigned)n_items), dim3(kWgSize), tf_lds_bytes(max_tf_k), s, slots_dev,
                     items_dev);
  return hipGetLastError();
}

}  // namespace vr
