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

// One pass over one view.  Each ray is marched by a pair of lanes (the group
// walk of the in-core kernel, resumed at each ray's saved index), a
// workgroup covers half a 16x16 super-tile, taken centre-out when the launch
// carries the in-core kernel's super-tile order (the tiles whose rays cross
// the most volume first), else in Morton-chunk order: samples in empty
// bricks are leapt over, samples in resident bricks evaluated from their
// slot, and a ray parks at its first sample in an occupied brick of a later
// pass (the sample is not composited; the ray resumes there).
// state: per pixel (C_r, C_g, C_b, T); next: the next lattice index, or -1
// once the ray is finished.  first: initialise the state instead of reading it.
// The LDS boxes allow three workgroups per CU; the register budget matches.
constexpr int kBrickRayGroup = 2;

template <int DT>
__global__ __launch_bounds__(kWgSize) __attribute__((amdgpu_waves_per_eu(3, 3))) void k_bricked_pass(
    const BrickedArgs args) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const BrickedArgs &a = kernarg<BrickedArgs>();
  int part;
  const SuperTile tile = group_tile_of<kBrickRayGroup>(a.order, blockIdx.x, a.W, a.H, 1, kDefaultChunkEdge, part);
  if (!tile.valid) return;  // uniform over the workgroup
  TfShared s = carve_tf(lds, a.tf.K);
  const bool tf_ok = load_tf(s, a.tf);
  int col, row;
  group_pixel_of<kBrickRayGroup>(tile.sx, tile.sy, part, col, row);
  const bool inside = col < a.W && row < a.H;
  const bool lead = (threadIdx.x % kBrickRayGroup) == 0;  // the lane that stores its ray's state
  const size_t pix = inside ? (size_t)row * a.W + col : 0;
  if (!tf_ok) {  // uniform: an invalid TF finishes every ray with NaN
    if (inside && lead) {
      a.state[pix] = nan_rgba();
      a.next[pix] = -1;
    }
    return;
  }
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
  const int S = a.slot_edge, E = a.vol.edge;
  // LDS value box of the wavefront, filled from one slot: the slot holds its
  // footprint edge-clamped, so within the slot's extent no further clamping
  // is needed and the box sees exactly the taps reconstruct_slot reads.
  ValBox box;
  box.valid = false;
  box.ox = box.oy = box.oz = 0;
  box.cells = a.use_box ? reinterpret_cast<float *>(lds + vbox_lds_offset(a.tf.K)) + (threadIdx.x / kWaveSize) * kVBoxCells
                        : nullptr;
  int box_slot = -1;  // uniform: the slot the box holds
  int step_brick = -1, step_slot = -1;  // this lane's brick and slot at the current step (prep -> eval)
  auto prep = [&](bool want, float px, float py, float pz) {
    step_brick = -1;
    step_slot = -1;
    if (want) {
      int bc[3];
      step_brick = block_of(a.vol, px, py, pz, bc);
      step_slot = a.page[step_brick];
    }
    if (!box.cells) return;
    const unsigned long long wm = __ballot(want);
    const int first = __ffsll((long long)wm) - 1;
    const int s0 = __builtin_amdgcn_readlane(step_slot, first);
    const int b0 = __builtin_amdgcn_readlane(step_brick, first);
    if (s0 < 0 || __ballot(want && step_slot != s0) != 0ull) {  // not one resident brick
      box.valid = false;
      return;
    }
    if (s0 != box_slot) box.valid = false;
    box_slot = s0;
    const int bx = b0 % a.vol.nbx, by = (b0 / a.vol.nbx) % a.vol.nby, bz = b0 / (a.vol.nbx * a.vol.nby);
    VolConst sv = a.vol;  // the slot as a small volume of S^3 voxels
    sv.nx = sv.ny = sv.nz = S;
    sv.bytes = (uint32_t)a.slot_bytes;
    const __amdgpu_buffer_rsrc_t srs = make_rsrc(a.pool + (size_t)s0 * a.slot_bytes, (uint32_t)a.slot_bytes);
    vbox_prepare<DT>(box, srs, sv, r, want, px - (float)(bx * E - 1), py - (float)(by * E - 1),
                     pz - (float)(bz * E - 1));
  };
  auto eval = [&](int, float px, float py, float pz) -> ChainSample {
    const int slot = step_slot;
    if (slot < 0) return ChainSample{0.0f, 0.0f, 0.0f, kStopSample};  // a later pass holds this brick
    int bc[3];
    block_of(a.vol, px, py, pz, bc);
    Stencil sten = make_stencil(px, py, pz);
    const int ox = bc[0] * E - 1, oy = bc[1] * E - 1, oz = bc[2] * E - 1;
    float val;
    if (box.valid) {  // every sampling lane is in the box's slot
      sten.ix -= ox;
      sten.iy -= oy;
      sten.iz -= oz;
      val = reconstruct_box(box, sten);
    } else {
      val = reconstruct_slot<DT>(a.pool + (size_t)slot * a.slot_bytes, S, ox, oy, oz, a.vol.nx, a.vol.ny, a.vol.nz,
                                 sten);
    }
    const Classified q = classify(s, a.tf.K, a.tf.v0, a.tf.scale, val);
    return ChainSample{q.c.x, q.c.y, q.c.z, transmit(q.c.w, sl2)};
  };
  auto take = [](bool, const ChainState &) {};
  NoFlat flat;
  NoPost post;
  // skipping on the fine blocks; the brick of a sample to evaluate decides
  // whether this pass has it
  const int parked = walk_group<kBrickRayGroup, false, true>(a.fine, s, a.tf, a.mc, r, eval, prep, take, flat, post,
                                                              st, kstart);
  if (active && lead) {
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

hipError_t launch_bricked_pass(const BrickedArgs &a0, hipStream_t s) {
  BrickedArgs a = a0;
  const int tiles = ((a.W + kSuperEdge - 1) / kSuperEdge) * ((a.H + kSuperEdge - 1) / kSuperEdge);
  uint32_t lds = tf_lds_bytes(a.tf.K);
  const uint32_t with_box = vbox_lds_offset(a.tf.K) + vbox_lds_bytes();
  a.use_box = with_box <= max_lds_per_workgroup() ? 1 : 0;
  if (a.use_box) lds = with_box;
  const void *fn = a.vol.dtype == kU16   ? reinterpret_cast<const void *>(&k_bricked_pass<kU16>)
                   : a.vol.dtype == kI16 ? reinterpret_cast<const void *>(&k_bricked_pass<kI16>)
                                         : reinterpret_cast<const void *>(&k_bricked_pass<kF32>);
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  const int64_t grid = group_grid(a.order ? (int64_t)tiles : grid_size_for(a.W, a.H, 1, kDefaultChunkEdge), kBrickRayGroup);
  switch (a.vol.dtype) {
  case kU16: hipLaunchKernelGGL(k_bricked_pass<kU16>, dim3((unsigned)grid), dim3(kWgSize), lds, s, a); break;
  case kI16: hipLaunchKernelGGL(k_bricked_pass<kI16>, dim3((unsigned)grid), dim3(kWgSize), lds, s, a); break;
  default: hipLaunchKernelGGL(k_bricked_pass<kF32>, dim3((unsigned)grid), dim3(kWgSize), lds, s, a); break;
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
