// render_bwd.hip -- adjoint of the forward ray caster (gfx950).
//
// Forward model per ray: C = sum_k T_k a_k c_k, T_{k+1} = T_k (1 - a_k),
// A = 1 - T_end, a_k = 1 - exp(-sigma_k step).  For L with g = dL/d(C, A):
//   dL/dc_k     = g_C T_k a_k
//   dL/dsigma_k = step (g_C . (T_{k+1} c_k - S_k) + g_A T_end),
//   S_k = sum_{m>k} T_m a_m c_m = C_end - C_{<=k},
// then through the TF segment (node difference x (K-1)/(v1-v0), zero where u
// was clamped) to the value, and through the 64 B-spline weights to the
// voxels.  The march is recomputed front to back with the forward's exact
// arithmetic, so C_{<=k}, T_k and the early-termination sample are the
// forward's; C_end and T_end come from the saved forward image.  Nothing per
// sample is stored.
#include "vr_internal.h"

namespace vr {

// dv * w_a w_b w_c onto the 64 taps (clamped taps pile onto edge voxels).
__device__ inline void scatter_taps(float *g, const VolConst &v, const Stencil &st, float dv) {
  int xs[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) xs[a] = min(max(st.ix - 1 + a, 0), v.nx - 1);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    uint32_t z = (uint32_t)min(max(st.iz - 1 + c, 0), v.nz - 1);
    float wc = dv * st.wz[c];
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      uint32_t y = (uint32_t)min(max(st.iy - 1 + b, 0), v.ny - 1);
      uint32_t rowb = (z * (uint32_t)v.ny + y) * (uint32_t)v.nx;
      float wb = wc * st.wy[b];
#pragma unroll
      for (int a = 0; a < 4; ++a) unsafeAtomicAdd(g + rowb + (uint32_t)xs[a], wb * st.wx[a]);
    }
  }
}

template <int DT>
__device__ inline void march_backward(const VolConst &v, const TfShared &s, float *sgtf, const TfConst &tf,
                                      const MarchConst &mc, const Ray &r, __amdgpu_buffer_rsrc_t rs, float4 g,
                                      float4 fin, float *grad_vol) {
  float C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, T = 1.0f;
  const float sl2 = mc.step * 1.4426950408889634f;
  const bool ert_on = mc.ert > 0.0f && mc.ert < 1.0f;
  const float Tend = 1.0f - fin.w;
  auto visit = [&](int, float px, float py, float pz) -> bool {
    Stencil st = make_stencil(px, py, pz);
    float val = reconstruct<DT>(rs, v, st);
    Classified q = classify(s, tf.K, tf.v0, tf.scale, val);
    float e = transmit(q.c.w, sl2);
    float ta = T * (1.0f - e);  // T_k a_k
    C0 = fmaf(ta, q.c.x, C0);
    C1 = fmaf(ta, q.c.y, C1);
    C2 = fmaf(ta, q.c.z, C2);
    T = T * e;  // T_{k+1}
    // adjoint of sample k
    float dc0 = g.x * ta, dc1 = g.y * ta, dc2 = g.z * ta;
    float acc = g.w * Tend;
    acc = fmaf(g.x, T * q.c.x - (fin.x - C0), acc);
    acc = fmaf(g.y, T * q.c.y - (fin.y - C1), acc);
    acc = fmaf(g.z, T * q.c.z - (fin.z - C2), acc);
    float dsig = mc.step * acc;
    if (sgtf) {
      float w1 = q.w, w0 = 1.0f - q.w;
      float *n0 = sgtf + 4 * q.j;
      atomicAdd(n0 + 0, w0 * dc0);
      atomicAdd(n0 + 1, w0 * dc1);
      atomicAdd(n0 + 2, w0 * dc2);
      atomicAdd(n0 + 3, w0 * dsig);
      atomicAdd(n0 + 4, w1 * dc0);
      atomicAdd(n0 + 5, w1 * dc1);
      atomicAdd(n0 + 6, w1 * dc2);
      atomicAdd(n0 + 7, w1 * dsig);
    }
    if (grad_vol && !q.clamped) {
      float4 a = s.node[q.j], b = s.node[q.j + 1];
      float dv = dc0 * (b.x - a.x);
      dv = fmaf(dc1, b.y - a.y, dv);
      dv = fmaf(dc2, b.z - a.z, dv);
      dv = fmaf(dsig, b.w - a.w, dv);
      dv *= tf.scale;
      if (dv != 0.0f) scatter_taps(grad_vol, v, st, dv);
    }
    return !(ert_on && (1.0f - T) >= mc.ert);
  };
  walk(v, s, tf, mc, r, visit);
}

template <int DT>
__global__ __launch_bounds__(kWgSize) void k_render_bwd(const BackwardArgs args) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const BackwardArgs &a = kernarg<BackwardArgs>();
  const RenderArgs &ra = a.r;
  SuperTile st = map_workgroup(blockIdx.x, ra.W, ra.H, ra.n_views, ra.chunk_edge);
  if (!st.valid) return;  // uniform over the workgroup
  const int K = ra.tf.K;
  float *sgtf = a.grad_tf ? reinterpret_cast<float *>(lds + tf_lds_bytes(K)) : nullptr;
  if (sgtf)
    for (int j = threadIdx.x; j < 4 * K; j += kWgSize) sgtf[j] = 0.0f;
  TfShared s = carve_tf(lds, K);
  load_tf(s, ra.tf);  // ends with a barrier, which also orders the zeroing
  int col, row;
  pixel_of(st.sx, st.sy, col, row);
  // every lane enters the march (it steps the wavefront in unison); lanes
  // outside the image or without a gradient carry an empty ray
  Ray r;
  r.hit = false;
  r.ns = 0;
  r.k0 = 0;
  float4 g = make_float4(0.0f, 0.0f, 0.0f, 0.0f), fin = g;
  if (col < ra.W && row < ra.H) {
    size_t pix = ((size_t)st.view * ra.H + row) * ra.W + col;
    g = reinterpret_cast<const float4 *>(a.grad_rgba)[pix];
    if (g.x != 0.0f || g.y != 0.0f || g.z != 0.0f || g.w != 0.0f) {
      r = setup_ray(ra.cams[st.view], col, row, ra.vol.nx, ra.vol.ny, ra.vol.nz, ra.mc.step);
      fin = reinterpret_cast<const float4 *>(a.out_rgba)[pix];
    }
  }
  __amdgpu_buffer_rsrc_t rs = make_rsrc(ra.vol.data, ra.vol.bytes);
  march_backward<DT>(ra.vol, s, sgtf, ra.tf, ra.mc, r, rs, g, fin, a.grad_vol);
  if (sgtf) {
    __syncthreads();
    for (int j = threadIdx.x; j < 4 * K; j += kWgSize) {
      float val = sgtf[j];
      if (val != 0.0f) unsafeAtomicAdd(a.grad_tf + j, val);
    }
  }
}

hipError_t launch_render_backward(const BackwardArgs &a, hipStream_t s) {
  const RenderArgs &ra = a.r;
  int64_t grid = grid_size_for(ra.W, ra.H, ra.n_views, ra.chunk_edge);
  uint32_t lds = tf_lds_bytes(ra.tf.K) + (a.grad_tf ? (uint32_t)ra.tf.K * 16u : 0u);
  switch (ra.vol.dtype) {
  case kU16: hipLaunchKernelGGL(k_render_bwd<kU16>, dim3((unsigned)grid), dim3(kWgSize), lds, s, a); break;
  case kI16: hipLaunchKernelGGL(k_render_bwd<kI16>, dim3((unsigned)grid), dim3(kWgSize), lds, s, a); break;
  case kF32: hipLaunchKernelGGL(k_render_bwd<kF32>, dim3((unsigned)grid), dim3(kWgSize), lds, s, a); break;
  default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace vr
