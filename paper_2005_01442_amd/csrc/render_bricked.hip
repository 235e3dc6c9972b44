// render_bricked.hip -- out-of-core rendering passes over a device brick pool
// (gfx950).
//
// The paper decomposes volumes larger than GPU memory into overlapping blocks
// and renders them block by block, front to back (Section 2: block
// decomposition, the overlap of three voxels for cubic sampling, Fig. 3, and
// the analysis of its pros and cons).  Here a brick is one block's footprint
// [bE-1, bE+E+1] per axis (the voxels any sample whose cell lies in the block
// reads, edge-clamped), resident in a pool slot of (E+3)^3 voxels.  A pass
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
  const bool xrow = DT != kF32 && s.ix >= 1 && s.ix + 2 <= nx - 1;  // the 4 x taps are one contiguous run
  int xs[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) xs[a] = min(max(s.ix - 1 + a, 0), nx - 1) - ox;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const int z = min(max(s.iz - 1 + c, 0), nz - 1) - oz;
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int y = min(max(s.iy - 1 + b, 0), ny - 1) - oy;
      const size_t row = ((size_t)z * S + y) * S;
      if (xrow) {
        // 16-bit taps: the dword-aligned 12-byte window holding them, shifted
        // by the run's parity (the slot padding keeps the window inside)
        const size_t e = row + xs[0];
        const uint32_t *w = reinterpret_cast<const uint32_t *>(slot + (e & ~(size_t)1) * 2);
        const uint32_t sh = (uint32_t)(e & 1) * 16u;
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
        continue;
      }
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        const size_t e = row + xs[a];
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

// One pass over one view.  One lane per pixel (16x16 pixels per workgroup,
// row-major over the image).  state: per pixel (C_r, C_g, C_b, T); next: the
// next lattice index, or -1 once the ray is finished.  first: initialise the
// state instead of reading it.
template <int DT>
__global__ __launch_bounds__(kWgSize) void k_bricked_pass(const BrickedArgs args) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const BrickedArgs &a = kernarg<BrickedArgs>();
  TfShared s = carve_tf(lds, a.tf.K);
  load_tf(s, a.tf);
  const int tiles_x = (a.W + kSuperEdge - 1) / kSuperEdge;
  const int col = (int)(blockIdx.x % tiles_x) * kSuperEdge + (int)(threadIdx.x % kSuperEdge);
  const int row = (int)(blockIdx.x / tiles_x) * kSuperEdge + (int)(threadIdx.x / kSuperEdge);
  if (col >= a.W || row >= a.H) return;
  const size_t pix = (size_t)row * a.W + col;
  int k;
  float4 st;
  if (a.first) {
    k = 0;
    st = make_float4(0.0f, 0.0f, 0.0f, 1.0f);
  } else {
    k = a.next[pix];
    if (k < 0) return;
    st = a.state[pix];
  }
  const Ray r = setup_ray(a.cam, col, row, a.vol.nx, a.vol.ny, a.vol.nz, a.mc.step);
  if (a.first) k = r.k0;
  const int kend = r.hit ? r.k0 + r.ns : 0;
  const float sl2 = a.mc.step * 1.4426950408889634f;
  const bool ert_on = a.mc.ert > 0.0f && a.mc.ert < 1.0f;
  const int S = a.slot_edge;
  bool done = !r.hit;
  int bc[3];
  while (!done && k < kend) {
    float px, py, pz;
    lattice_point(r, a.mc.step, k, px, py, pz);
    const int b = block_of(a.vol, px, py, pz, bc);
    if (!a.occ[b]) {  // empty brick: its samples add exactly zero
      const int t = leap_target(a.vol, r, bc, a.mc.step, k);
      k = t > k + 1 ? t : k + 1;
      continue;
    }
    const int slot = a.page[b];
    if (slot < 0) break;  // a later pass holds this brick
    const Stencil sten = make_stencil(px, py, pz);
    const char *base = a.pool + (size_t)slot * a.slot_bytes;
    const int E = a.vol.edge;
    const float val = reconstruct_slot<DT>(base, S, bc[0] * E - 1, bc[1] * E - 1, bc[2] * E - 1, a.vol.nx, a.vol.ny,
                                           a.vol.nz, sten);
    const Classified q = classify(s, a.tf.K, a.tf.v0, a.tf.scale, val);
    const float e = transmit(q.c.w, sl2);
    const float ta = st.w * (1.0f - e);
    st.x = fmaf(ta, q.c.x, st.x);
    st.y = fmaf(ta, q.c.y, st.y);
    st.z = fmaf(ta, q.c.z, st.z);
    st.w = st.w * e;
    ++k;
    if (ert_on && (1.0f - st.w) >= a.mc.ert) done = true;
  }
  if (k >= kend) done = true;
  a.state[pix] = st;
  a.next[pix] = done ? -1 : k;
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
