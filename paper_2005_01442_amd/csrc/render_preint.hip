// render_preint.hip -- pre-integrated classification (gfx950).
//
// The paper pairs its ray caster with tables of previously integrated
// rendering (Section 2, the proposed method; the conclusion names
// pre-integrated rendering against sampling artefacts).  A ray segment of one
// step along which the value rises linearly from TF node i to node j has the
// emission-absorption integrals
//   alpha = 1 - exp(-tau(step)),  C = integral c(u(x)) sigma(u(x)) exp(-tau(x)) dx,
// tau(x) = integral_0^x sigma(u(x')) dx', u(x) = i + (j - i) x / step.
// k_preint_table tabulates them for every node pair; k_render_preint walks
// the lattice cells (between the boundaries t = k step and (k+1) step, the
// cells whose midpoints are the post-classified samples), reconstructs the
// value at each boundary once, and composites each cell with the table's
// bilinear lookup at (u(front), u(back)).
#include "vr_internal.h"

namespace vr {

// ---------------------------------------------------------------------------
// Table: one thread per entry, FP64.  The segment is split where u crosses a
// node (sigma and c are linear between); each piece into sub-intervals of
// optical depth <= 1/32, each integrated with 4-point Gauss-Legendre, tau
// exact (the integral of a linear sigma); stop once tau > 60.
// ---------------------------------------------------------------------------
__device__ inline void tf_node(const float *tf, int K, int j, double out[4]) {
  j = min(max(j, 0), K - 1);
  const float4 n = reinterpret_cast<const float4 *>(tf)[j];
  out[0] = n.x;
  out[1] = n.y;
  out[2] = n.z;
  out[3] = n.w;  // the table kernel has checked every node
}

__global__ __launch_bounds__(256) void k_preint_table(const float *tf, int K, double step, float4 *out,
                                                     uint32_t *status) {
  // an invalid node anywhere makes the whole table NaN (and is recorded)
  int bad = 0;
  for (int j = threadIdx.x; j < K; j += 256) bad |= tf_node_valid(reinterpret_cast<const float4 *>(tf)[j]) ? 0 : 1;
  bad = __syncthreads_or(bad);
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (bad) {
    if (threadIdx.x == 0 && status) __hip_atomic_store(status, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (e < (int64_t)K * K) out[e] = nan_rgba();
    return;
  }
  if (e >= (int64_t)K * K) return;
  const int i = (int)(e / K), j = (int)(e % K);
  double C[3] = {0.0, 0.0, 0.0}, tau = 0.0;
  if (i == j) {
    double n[4];
    tf_node(tf, K, i, n);
    tau = n[3] * step;
    const double a = -expm1(-tau);
    for (int c = 0; c < 3; ++c) C[c] = n[c] * a;
  } else {
    const int n = abs(j - i), dir = j > i ? 1 : -1;
    const double piece = step / (double)n;
    // 4-point Gauss-Legendre on [-1, 1]
    const double gx[4] = {-0.8611363115940526, -0.3399810435848563, 0.3399810435848563, 0.8611363115940526};
    const double gw[4] = {0.3478548451374538, 0.6521451548625461, 0.6521451548625461, 0.3478548451374538};
    for (int m = 0; m < n && tau <= 60.0; ++m) {
      double ea[4], eb[4];
      tf_node(tf, K, i + dir * m, ea);
      tf_node(tf, K, i + dir * (m + 1), eb);
      const double ds = (eb[3] - ea[3]) / piece;  // d sigma / dx on this piece
      const double tau_piece = 0.5 * (ea[3] + eb[3]) * piece;
      const int sub = max(1, (int)ceil(tau_piece * 32.0));
      const double h = piece / (double)sub;
      for (int q = 0; q < sub; ++q) {
        const double x0 = q * h;
        if (tau + ea[3] * x0 + 0.5 * ds * x0 * x0 > 60.0) break;
        for (int g = 0; g < 4; ++g) {
          const double x = x0 + 0.5 * h * (1.0 + gx[g]);
          const double w = x / piece;
          const double sg = ea[3] + ds * x;
          const double f = 0.5 * h * gw[g] * sg * exp(-(tau + ea[3] * x + 0.5 * ds * x * x));
          for (int c = 0; c < 3; ++c) C[c] += ((1.0 - w) * ea[c] + w * eb[c]) * f;
        }
      }
      tau += tau_piece;
    }
  }
  out[e] = make_float4((float)C[0], (float)C[1], (float)C[2], (float)(-expm1(-tau)));
}

hipError_t launch_preint_table(const float *tf, int K, float step, float4 *out, uint32_t *status, hipStream_t s) {
  const int64_t n = (int64_t)K * K;
  hipLaunchKernelGGL(k_preint_table, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, tf, K, (double)step, out,
                     status);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Render.
// ---------------------------------------------------------------------------

// Bilinear lookup of the table at node coordinates (uf, ub), clamped.
__device__ inline float4 preint_lookup(const float4 *tab, int K, float uf, float ub) {
  uf = fminf(fmaxf(uf, 0.0f), (float)(K - 1));
  ub = fminf(fmaxf(ub, 0.0f), (float)(K - 1));
  const int i = min((int)uf, K - 2), j = min((int)ub, K - 2);
  const float wf = uf - (float)i, wb = ub - (float)j;
  const float4 *r0 = tab + (size_t)i * K + j;
  const float4 p00 = r0[0], p01 = r0[1], p10 = r0[K], p11 = r0[K + 1];
  float4 o;
  o.x = fmaf(wf, fmaf(wb, p11.x - p10.x, p10.x) - fmaf(wb, p01.x - p00.x, p00.x), fmaf(wb, p01.x - p00.x, p00.x));
  o.y = fmaf(wf, fmaf(wb, p11.y - p10.y, p10.y) - fmaf(wb, p01.y - p00.y, p00.y), fmaf(wb, p01.y - p00.y, p00.y));
  o.z = fmaf(wf, fmaf(wb, p11.z - p10.z, p10.z) - fmaf(wb, p01.z - p00.z, p00.z), fmaf(wb, p01.z - p00.z, p00.z));
  o.w = fmaf(wf, fmaf(wb, p11.w - p10.w, p10.w) - fmaf(wb, p01.w - p00.w, p00.w), fmaf(wb, p01.w - p00.w, p00.w));
  return o;
}

// Walk the boundary points k = k0 .. k0 + ns of a ray with the wavefront in
// step (as `walk` does for samples).  At point k > k0 the cell k - 1 closes.
// Skipping: a cell is skipped iff no value in the union of its two points'
// block ranges meets extinction (its ramp then integrates to exactly zero);
// a cell's front value is reused from the previous point when that point was
// reconstructed, else reconstructed first.  When no lane closes a cell the
// wavefront leaps (points up to the leap target stay in the current, empty,
// block, so every skipped cell lies in one empty block).
template <int DT>
__device__ inline float4 march_preint(const VolConst &v, const TfShared &s, const TfConst &tf, const MarchConst &mc,
                                      const float4 *tab, const Ray &r0, __amdgpu_buffer_rsrc_t rs, ValBox &box,
                                      uint32_t &evaluated, uint32_t &unstaged) {
  Ray r = r0;
  r.s0 = r0.s0 - 0.5f * mc.step;  // boundary point k sits at s0 + (k - k0) step - step/2
  const bool ert_on = mc.ert > 0.0f && mc.ert < 1.0f;
  const int kb = r.hit ? r.k0 : 0x7fffffff;
  const int ke = r.hit ? r.k0 + r.ns + 1 : 0;
  bool alive = r.hit;
  int k = wave_min_i32(kb);
  const int kend = wave_max_i32(ke);
  int kfree = kb;  // points below kfree: before the ray, or left in an empty block
  // the grid constants of the block lookup and leap pinned in scalar
  // registers, so the loop does not re-read them from the kernel arguments
  // (vector registers would exceed this kernel's budget)
  VolConst vg = v;
  {
    int a0 = __builtin_amdgcn_readfirstlane(vg.nx), a1 = __builtin_amdgcn_readfirstlane(vg.ny),
        a2 = __builtin_amdgcn_readfirstlane(vg.nz), a3 = __builtin_amdgcn_readfirstlane(vg.edge_shift),
        a4 = __builtin_amdgcn_readfirstlane(vg.nbx), a5 = __builtin_amdgcn_readfirstlane(vg.nby);
    asm volatile("" : "+s"(a0), "+s"(a1), "+s"(a2), "+s"(a3), "+s"(a4), "+s"(a5));
    vg.nx = a0;
    vg.ny = a1;
    vg.nz = a2;
    vg.edge_shift = a3;
    vg.nbx = a4;
    vg.nby = a5;
  }
  int cb = -1;
  bool cocc = false;
  int bc[3] = {0, 0, 0};
  int kprev = -0x7fffffff;
  float vprev = 0.0f;
  float C0 = 0.0f, C1 = 0.0f, C2 = 0.0f, T = 1.0f;
  auto value_at = [&](float px, float py, float pz) -> float {
    Stencil st = make_stencil(px, py, pz);
    if (box.valid) return reconstruct_box(box, st);
    ++unstaged;
    return reconstruct<DT>(rs, v, st);
  };
  while (k < kend) {
    const bool in = alive && k >= kfree && k < ke;
    bool want = false;
    // every lane computes its point and cell (as walk does), shared with the
    // box test and the stencil
    float px, py, pz;
    lattice_point(r, mc.step, k, px, py, pz);
    const int ix = (int)floorf(px), iy = (int)floorf(py), iz = (int)floorf(pz);
    if (in) {
      if (mc.skip) {
        const int b = block_of_cell(vg, ix, iy, iz, bc);
        bool pair = cocc;
        if (b != cb) {
          const int pb = cb;
          const bool pocc = cocc;
          cb = b;
          cocc = block_occupied(v, s, tf, b);
          // two empty blocks: the cell between them is empty only if the
          // union of their ranges is
          pair = cocc || pocc ||
                 (pb >= 0 && range_occupied(s, tf.K, tf.v0, tf.scale, fminf(v.minmax[pb].x, v.minmax[b].x),
                                            fmaxf(v.minmax[pb].y, v.minmax[b].y)));
        }
        want = k > kb && pair;
      } else {
        want = k > kb;
      }
    }
    if (__ballot(want) == 0ull) {
      int prop = 0x7fffffff;
      if (in) {
        if (mc.skip && !cocc) {
          kfree = leap_target(vg, r, bc, mc.step, k);
          prop = kfree;
        } else {
          prop = k + 1;
        }
      } else if (alive && k < ke) {
        prop = kfree;
      }
      const int m = wave_min_i32(prop);
      k = m > k + 1 ? m : k + 1;
      continue;
    }
    const bool need_front = want && kprev != k - 1;
    if (__ballot(need_front) != 0ull) {
      float fx = 0.0f, fy = 0.0f, fz = 0.0f;
      if (need_front) lattice_point(r, mc.step, k - 1, fx, fy, fz);
      if (box.cells) vbox_prepare<DT>(box, rs, v, r, need_front, fx, fy, fz);
      if (need_front) vprev = value_at(fx, fy, fz);
    }
    if (box.cells) vbox_prepare<DT>(box, rs, v, r, want, px, py, pz);
    if (want) {
      const float vcur = value_at(px, py, pz);
      const float4 q = preint_lookup(tab, tf.K, (vprev - tf.v0) * tf.scale, (vcur - tf.v0) * tf.scale);
      C0 = fmaf(T, q.x, C0);
      C1 = fmaf(T, q.y, C1);
      C2 = fmaf(T, q.z, C2);
      T = T * (1.0f - q.w);
      ++evaluated;
      vprev = vcur;
      kprev = k;
      if (ert_on && (1.0f - T) >= mc.ert) alive = false;
    }
    ++k;
  }
  return make_float4(C0, C1, C2, 1.0f - T);
}

// One wavefront item of the pre-integrated render: wavefront w (an 8x8
// sub-tile) of super-tile item i; n_items bounds the order.
template <int DT>
__device__ inline void preint_wave_item(const RenderArgs &a, const TfShared &s, bool tf_ok, const float4 *tab,
                                        ValBox &box, __amdgpu_buffer_rsrc_t rs, int64_t i, int w, int64_t n_items,
                                        uint32_t &evaluated, uint32_t &unstaged, uint32_t &lattice, uint32_t &hits) {
  if (a.order && i >= n_items) return;  // padding of the last queue
  const SuperTile st = tile_of(a.order, i, a.W, a.H, a.n_views, a.chunk_edge);
  if (!st.valid) return;  // uniform over the wavefront
  const int lane = (int)(threadIdx.x % kWaveSize);
  const int col = st.sx * kSuperEdge + (w & 1) * kTileEdge + (lane & 7);
  const int row = st.sy * kSuperEdge + (w >> 1) * kTileEdge + (lane >> 3);
  const bool inside = col < a.W && row < a.H;
  if (!tf_ok) {
    if (inside) reinterpret_cast<float4 *>(a.out)[((size_t)st.view * a.H + row) * a.W + col] = nan_rgba();
    return;
  }
  const CamConst &cam = a.cams[st.view];
  Ray r;
  r.hit = false;
  r.ns = 0;
  r.k0 = 0;
  r.s0 = 0.0f;
  if (inside) r = setup_ray(cam, col, row, a.vol.nx, a.vol.ny, a.vol.nz, a.mc.step);
  const float4 rgba = march_preint<DT>(a.vol, s, a.tf, a.mc, tab, r, rs, box, evaluated, unstaged);
  if (inside) reinterpret_cast<float4 *>(a.out)[((size_t)st.view * a.H + row) * a.W + col] = rgba;
  lattice += (uint32_t)r.ns;
  hits += r.hit ? 1u : 0u;
}

// Queued like the whole-image forward (one super-tile per workgroup without
// queue counters); registers budgeted for three wavefronts per SIMD, which
// the LDS value boxes allow.
template <int DT>
__global__ __launch_bounds__(kWgSize) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_render_preint(
    const RenderArgs args, const float4 *tab) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const RenderArgs &a = kernarg<RenderArgs>();
  const int64_t n_items = (int64_t)a.n_views * ((a.W + kSuperEdge - 1) / kSuperEdge) * ((a.H + kSuperEdge - 1) / kSuperEdge);
  if (!a.queue && !tile_of(a.order, blockIdx.x, a.W, a.H, a.n_views, a.chunk_edge).valid)
    return;  // uniform over the workgroup
  TfShared s = carve_tf(lds, a.tf.K);
  if (a.occ_lds_words > 0)
    stage_occupancy(s, a.vol, lds + vbox_lds_offset(a.tf.K) + vbox_lds_bytes(), a.occ_lds_words);
  const bool tf_ok = load_tf(s, a.tf);
  __amdgpu_buffer_rsrc_t rs = make_rsrc(a.vol.data, a.vol.bytes);
  ValBox box;
  box.valid = false;
  box.ox = box.oy = box.oz = 0;
  box.cells = a.use_box ? reinterpret_cast<float *>(lds + vbox_lds_offset(a.tf.K)) + (threadIdx.x / kWaveSize) * kVBoxCells
                        : nullptr;
  uint32_t evaluated = 0, unstaged = 0, lattice = 0, hits = 0;
  if (!a.queue) {
    preint_wave_item<DT>(a, s, tf_ok, tab, box, rs, blockIdx.x, (int)(threadIdx.x / kWaveSize), n_items, evaluated,
                         unstaged, lattice, hits);
  } else {
    const int x = (int)(blockIdx.x % kXcds);
    int w = 0;
    int64_t i = 0;
    while (next_wave_item(a.queue, (uint32_t)a.queue_items, x, i, w))
      preint_wave_item<DT>(a, s, tf_ok, tab, box, rs, i, w, n_items, evaluated, unstaged, lattice, hits);
  }
  if (a.counters) {
    wave_count(a.counters + 0, evaluated);
    wave_count(a.counters + 1, lattice);
    wave_count(a.counters + 2, hits);
    wave_count(a.counters + 3, unstaged);
  }
}

hipError_t launch_render_preint(const RenderArgs &a0, const float4 *tab, hipStream_t s) {
  RenderArgs a = a0;
  int64_t grid = render_grid(a);
  uint32_t lds = tf_lds_bytes(a.tf.K);
  const uint32_t with_box = vbox_lds_offset(a.tf.K) + vbox_lds_bytes();
  a.use_box = with_box <= max_lds_per_workgroup() ? 1 : 0;
  if (a.use_box) lds = with_box;
  a.occ_lds_words = occupancy_lds_words(a, lds);
  lds += (uint32_t)a.occ_lds_words * 4u;
  const void *fn = a.vol.dtype == kU16   ? reinterpret_cast<const void *>(&k_render_preint<kU16>)
                   : a.vol.dtype == kI16 ? reinterpret_cast<const void *>(&k_render_preint<kI16>)
                                         : reinterpret_cast<const void *>(&k_render_preint<kF32>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  a.queue = nullptr;
  a.queue_items = 0;
  if (a.order) {
    const int64_t resident = resident_workgroups(fn, lds);
    const int64_t padded = (grid + kXcds - 1) / kXcds * kXcds;  // queue i mod 8 holds items i
    if (resident >= kXcds && resident < grid) {
      a.queue = reinterpret_cast<uint32_t *>(const_cast<int32_t *>(a.order) + tile_order_count(a));
      a.queue_items = (int32_t)(padded / kXcds * kWavesPerWg);
      grid = resident;
    }
  }
  switch (a.vol.dtype) {
  case kU16: hipLaunchKernelGGL(k_render_preint<kU16>, dim3((unsigned)grid), dim3(kWgSize), lds, s, a, tab); break;
  case kI16: hipLaunchKernelGGL(k_render_preint<kI16>, dim3((unsigned)grid), dim3(kWgSize), lds, s, a, tab); break;
  default: hipLaunchKernelGGL(k_render_preint<kF32>, dim3((unsigned)grid), dim3(kWgSize), lds, s, a, tab); break;
  }
  return hipGetLastError();
}

}  // namespace vr
