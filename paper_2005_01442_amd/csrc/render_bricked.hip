// render_bricked.hip -- out-of-core rendering passes over a device brick pool
// (gfx950).
//
// The paper decomposes volumes larger than GPU memory into overlapping blocks
// and renders them block by block, front to back (Section 2: block
// decomposition, the overlap of three voxels for cubic sampling, Fig. 3, and
// the analysis of its pros and cons).  Here a brick is one block's footprint
// [bE-1, bE+E+1] per axis (the voxels any sample whose cell lies in the block
// reads, edge-clamped; one more plane per axis makes the slot edge E+4 even),
// resident in a pool slot of (E+4)^3 voxels.  A pass
// renders, for every ray, its samples in the resident bricks, continuing from
// the ray's state (next lattice index, C, T) that earlier passes left; passes
// follow a front-to-back brick order, so every ray's samples are composited
// in lattice order and the image equals the in-core render with skipping
// bit for bit.
#include "vr_internal.h"

namespace vr {

// Value of a sample from its brick's slot: taps clamped to the grid, then
// addressed relative to the footprint origin (bE-1 per axis); the FMA order
// of every other reconstruction path.
template <int DT>
__device__ inline float reconstruct_slot(const char *slot, int S, int ox, int oy, int oz, int nx, int ny, int nz,
                                         const Stencil &s) {
  float t[4][4][4];
  const bool inner = (s.ix >= 1) & (s.ix + 2 <= nx - 1) & (s.iy >= 1) & (s.iy + 2 <= ny - 1) & (s.iz >= 1) &
                     (s.iz + 2 <= nz - 1);
  if (DT != kF32 && inner) {
    // 16-bit taps, no clamping: every x-run of 4 taps lies in the dword window
    // w0 + (c S + b) S / 2 .. + 2 (S is even, so all runs share e's parity;
    // the slot padding keeps the last window inside)
    const uint32_t e = ((uint32_t)(s.iz - 1 - oz) * (uint32_t)S + (uint32_t)(s.iy - 1 - oy)) * (uint32_t)S +
                       (uint32_t)(s.ix - 1 - ox);
    const uint32_t *w0 = reinterpret_cast<const uint32_t *>(slot) + (e >> 1);
    const uint32_t sh = (e & 1u) * 16u, half = (uint32_t)S >> 1;
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const uint32_t *w = w0 + ((uint32_t)c * (uint32_t)S + (uint32_t)b) * half;
        const uint32_t lo = __builtin_amdgcn_alignbit(w[1], w[0], sh), hi = __builtin_amdgcn_alignbit(w[2], w[1], sh);
        if (DT == kI16) {
          t[c][b][0] = (float)(int16_t)(lo & 0xffffu);
          t[c][b][1] = (float)((int32_t)lo >> 16);
          t[c][b][2] = (float)(int16_t)(hi & 0xffffu);
          t[c][b][3] = (float)((int32_t)hi >> 16);
        } else {
          t[c][b][0] = (float)(lo & 0xffffu);
          t[c][b][1] = (float)(lo >> 16);
          t[c][b][2] = (float)(hi & 0xffffu);
          t[c][b][3] = (float)(hi >> 16);
        }
      }
    return combine(s, t);
  }
  int xs[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) xs[a] = min(max(s.ix - 1 + a, 0), nx - 1) - ox;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int z = min(max(s.iz - 1 + c, 0), nz - 1) - oz;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int y = min(max(s.iy - 1 + b, 0), ny - 1) - oy;
      const uint32_t row = ((uint32_t)z * (uint32_t)S + (uint32_t)y) * (uint32_t)S;
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const uint32_t e = row + (uint32_t)xs[a];
        if (DT == kF32)
          t[c][b][a] = reinterpret_cast<const float *>(slot)[e];
        else if (DT == kI16)
          t[c][b][a] = (float)reinterpret_cast<const int16_t *>(slot)[e];
        else
          t[c][b][a] = (float)reinterpret_cast<const uint16_t *>(slot)[e];
      }
    }
  }
  return combine(s, t);
}

// One pass over one view.  Workgroups of 16x16 pixels in raster order,
// wavefronts of 8x8 that march their rays in step (the walk of the in-core
// kernel, started at each ray's saved index): samples in empty bricks are
// leapt over, samples in resident bricks evaluated from their slot, and a
// ray parks at its first sample in an occupied brick of a later pass.
// state: per pixel (C_r, C_g, C_b, T); next: the next lattice index, or -1
// once the ray is finished.  first: initialise the state instead of reading it.
template <int DT>
__global__ __launch_bounds__(kWgSize) void k_bricked_pass(const BrickedArgs args) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const BrickedArgs &a = kernarg<BrickedArgs>();
  TfShared s = carve_tf(lds, a.tf.K);
  load_tf(s, a.tf);
  const int tiles_x = (a.W + kSuperEdge - 1) / kSuperEdge;
  int col, row;
  pixel_of((int)(blockIdx.x % tiles_x), (int)(blockIdx.x / tiles_x), col, row);
  const bool inside = col < a.W && row < a.H;
  const size_t pix = inside ? (size_t)row * a.W + col : 0;
  int kstart = 0;
  float4 st = make_float4(0.0f, 0.0f, 0.0f, 1.0f);
  bool active = inside;
  if (inside && !a.first) {
    kstart = a.next[pix];
    active = kstart >= 0;
    if (active) st = a.state[pix];
  }
  // every lane takes part in the walk; finished or outside lanes carry no ray
  Ray r;
  r.hit = false;
  r.ns = 0;
  r.k0 = 0;
  r.s0 = 0.0f;
  if (active) r = setup_ray(a.cam, col, row, a.vol.nx, a.vol.ny, a.vol.nz, a.mc.step);
  if (a.first) kstart = r.k0;
  const float sl2 = a.mc.step * 1.4426950408889634f;
  const bool ert_on = a.mc.ert > 0.0f && a.mc.ert < 1.0f;
  const int S = a.slot_edge, E = a.vol.edge;
  int parked = -1;
  auto visit = [&](int k, float px, float py, float pz) -> bool {
    int bc[3];
    const int b = block_of(a.vol, px, py, pz, bc);
    const int slot = a.page[b];
    if (slot < 0) {  // a later pass holds this brick
      parked = k;
      return false;
    }
    const Stencil sten = make_stencil(px, py, pz);
    const float val = reconstruct_slot<DT>(a.pool + (size_t)slot * a.slot_bytes, S, bc[0] * E - 1, bc[1] * E - 1,
                                           bc[2] * E - 1, a.vol.nx, a.vol.ny, a.vol.nz, sten);
    const Classified q = classify(s, a.tf.K, a.tf.v0, a.tf.scale, val);
    const float e = transmit(q.c.w, sl2);
    const float ta = st.w * (1.0f - e);
    st.x = fmaf(ta, q.c.x, st.x);
    st.y = fmaf(ta, q.c.y, st.y);
    st.z = fmaf(ta, q.c.z, st.z);
    st.w = st.w * e;
    return !(ert_on && (1.0f - st.w) >= a.mc.ert);
  };
  NoPrep prep;
  NoPost post;
  // skipping on the fine blocks; the brick of a sample to evaluate decides
  // whether this pass has it
  walk<decltype(visit), NoPrep, NoPost, true>(a.fine, s, a.tf, a.mc, r, visit, prep, post, kstart);
  if (active) {
    a.state[pix] = st;
    a.next[pix] = parked;
  }
}

// Premultiplied RGBA from the pass state: (C, 1 - T).
__global__ __launch_bounds__(kWgSize) void k_bricked_finish(const float4 *state, float4 *out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kWgSize + threadIdx.x;
  if (i < n) {
    const float4 st = state[i];
    out[i] = make_float4(st.x, st.y, st.z, 1.0f - st.w);
  }
}

hipError_t launch_bricked_pass(const BrickedArgs &a, hipStream_t s) {
  const int tiles = ((a.W + kSuperEdge - 1) / kSuperEdge) * ((a.H + kSuperEdge - 1) / kSuperEdge);
  const uint32_t lds = tf_lds_bytes(a.tf.K);
  switch (a.vol.dtype) {
  case kU16: hipLaunchKernelGGL(k_bricked_pass<kU16>, dim3((unsigned)tiles), dim3(kWgSize), lds, s, a); break;
  case kI16: hipLaunchKernelGGL(k_bricked_pass<kI16>, dim3((unsigned)tiles), dim3(kWgSize), lds, s, a); break;
  default: hipLaunchKernelGGL(k_bricked_pass<kF32>, dim3((unsigned)tiles), dim3(kWgSize), lds, s, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_bricked_finish(const float4 *state, float4 *out, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_bricked_finish, dim3((unsigned)((n + kWgSize - 1) / kWgSize)), dim3(kWgSize), 0, s, state, out,
                     n);
  return hipGetLastError();
}

}  // namespace vr
