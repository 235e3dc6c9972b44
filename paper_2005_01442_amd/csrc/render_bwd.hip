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
#include <algorithm>

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

// ---------------------------------------------------------------------------
// Gradient box: each wavefront accumulates its grid-gradient scatter in a
// kBox^3 fp32 box of LDS placed over the slab its lanes are sampling; when a
// step's stencils leave the box, the box is flushed to global memory (one
// atomic per touched voxel) and re-placed.  Steps whose stencils spread wider
// than the box scatter straight to global memory.
// ---------------------------------------------------------------------------
constexpr int kBox = 14;   // box extent per axis
constexpr int kBoxY = 16;  // y stride
// z stride: with y stride 16 and z stride 228 the 64 taps a + 16 b + 228 c
// (a, b, c < 4) of one stencil fall in 64 distinct LDS banks
constexpr int kBoxZ = kBoxY * kBox + 4;
constexpr int kBoxCells = kBox * kBoxZ;
constexpr int kRec = 16;  // dwords per staged scatter record

// LDS layout of the adjoint: TF + prefix counts, TF gradient (4K floats per
// copy, when requested), then 16-byte aligned per-wavefront boxes and record
// areas.  Two copies of the TF gradient still leave two workgroups per CU.
constexpr int kTfGradCopies = 2;
__host__ __device__ inline uint32_t box_lds_offset(int K, bool with_tf_grad) {
  uint32_t o = tf_lds_bytes(K) + (with_tf_grad ? (uint32_t)K * 16u * kTfGradCopies : 0u);
  return (o + 15u) & ~15u;
}

struct GradBox {
  float *cells;  // this wavefront's LDS cells, [z][y][x], zero outside use
  float *recs;   // this wavefront's staged scatter records, kRec dwords per slot
  int ox, oy, oz;
  bool valid;
};

__device__ inline void box_flush(GradBox &b, float *grad, const VolConst &v) {
  if (!b.valid) return;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const int lane = threadIdx.x % kWaveSize;
  for (int i = lane; i < kBox * kBox * kBox; i += kWaveSize) {
    const int cx = i % kBox, cy = (i / kBox) % kBox, cz = i / (kBox * kBox);
    const int cell = cz * kBoxZ + cy * kBoxY + cx;
    float val = b.cells[cell];
    if (val != 0.0f) {
      int x = b.ox + cx, y = b.oy + cy, z = b.oz + cz;
      if (x < v.nx && y < v.ny && z < v.nz)
        unsafeAtomicAdd(grad + ((uint32_t)z * (uint32_t)v.ny + (uint32_t)y) * (uint32_t)v.nx + (uint32_t)x, val);
      b.cells[cell] = 0.0f;
    }
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  b.valid = false;
}

// Wavefront-wide: make the box cover every clamped stencil of this step's
// sampling lanes, if they fit.
__device__ inline void box_prepare(GradBox &b, float *grad, const VolConst &v, const Ray &r, bool want, float px,
                                   float py, float pz) {
  int lo[3] = {0x7fffffff, 0x7fffffff, 0x7fffffff}, hi[3] = {-1, -1, -1};
  const int n[3] = {v.nx, v.ny, v.nz};
  if (want) {
    const float p[3] = {px, py, pz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      int f = (int)floorf(p[a]);
      lo[a] = min(max(f - 1, 0), n[a] - 1);
      hi[a] = min(max(f + 2, 0), n[a] - 1);
    }
  }
  const int o[3] = {b.ox, b.oy, b.oz};
  bool inside = true;
  if (want)
#pragma unroll
    for (int a = 0; a < 3; ++a) inside = inside && lo[a] >= o[a] && hi[a] < o[a] + kBox;
  if (b.valid && __ballot(!inside) == 0ull) return;
  box_flush(b, grad, v);
  int mn[3], mx[3];
  bool fits = true;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    mn[a] = wave_min_i32(lo[a]);
    mx[a] = wave_max_i32(hi[a]);
    fits = fits && (mx[a] - mn[a] < kBox);
  }
  if (!fits) return;  // this step scatters to global memory
  // extend the box along the marching direction of the first sampling lane
  const unsigned long long wm = __ballot(want);
  const int first = __ffsll((long long)wm) - 1;
  int org[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    const float da = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, r.d[a]), first));
    int oa = da >= 0.0f ? mn[a] : mx[a] - kBox + 1;
    org[a] = max(oa, 0);
  }
  b.ox = __builtin_amdgcn_readfirstlane(org[0]);
  b.oy = __builtin_amdgcn_readfirstlane(org[1]);
  b.oz = __builtin_amdgcn_readfirstlane(org[2]);
  b.valid = true;
}

// A lane whose stencil is interior stages its scatter record (x, y, z weights
// with dv folded into the z weights, the box cell of tap (0, 0, 0) and its
// coordinates); the wavefront then applies the staged records with the lanes
// transposed onto the 64 taps (box_apply).  Clamped stencils, whose taps can
// coincide, add their taps with LDS atomics right away.
__device__ inline bool box_stage(GradBox &b, const VolConst &v, const Stencil &st, float dv) {
  const bool inner = (st.ix >= 1) & (st.ix + 2 <= v.nx - 1) & (st.iy >= 1) & (st.iy + 2 <= v.ny - 1) &
                     (st.iz >= 1) & (st.iz + 2 <= v.nz - 1);
  if (inner) {
    // records are packed in lane order: this lane's slot is its rank among
    // the staging lanes (all of which are active here together)
    const unsigned long long act = __ballot(1);
    const int rank = __builtin_amdgcn_mbcnt_hi((uint32_t)(act >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)act, 0u));
    float *rec = b.recs + rank * kRec;
    f32x4 wx = {st.wx[0], st.wx[1], st.wx[2], st.wx[3]};
    f32x4 wy = {st.wy[0], st.wy[1], st.wy[2], st.wy[3]};
    f32x4 wz = {dv * st.wz[0], dv * st.wz[1], dv * st.wz[2], dv * st.wz[3]};
    *reinterpret_cast<f32x4 *>(rec + 0) = wx;
    *reinterpret_cast<f32x4 *>(rec + 4) = wy;
    *reinterpret_cast<f32x4 *>(rec + 8) = wz;
    // box coordinates of tap (0, 0, 0): its cell, and two packings used to
    // find where two records' stencils overlap
    const int x = st.ix - 1 - b.ox, y = st.iy - 1 - b.oy, z = st.iz - 1 - b.oz;
    int4 m;
    m.x = z * kBoxZ + y * kBoxY + x;
    m.y = x + 16 * y + 256 * z;
    m.z = 4 * (x + 4 * y + 16 * z);
    m.w = 0;
    *reinterpret_cast<int4 *>(rec + 12) = m;
    return true;
  }
  int xs[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) xs[a] = min(max(st.ix - 1 + a, 0), v.nx - 1) - b.ox;
  for (int c = 0; c < 4; ++c) {
    int z = min(max(st.iz - 1 + c, 0), v.nz - 1) - b.oz;
    float wc = dv * st.wz[c];
    for (int bb = 0; bb < 4; ++bb) {
      int y = min(max(st.iy - 1 + bb, 0), v.ny - 1) - b.oy;
      float wb = wc * st.wy[bb];
#pragma unroll
      for (int a = 0; a < 4; ++a) atomicAdd(b.cells + z * kBoxZ + y * kBoxY + xs[a], wb * st.wx[a]);
    }
  }
  return false;
}

// Wavefront-wide: apply the records of the lanes in `staged` (packed in slots
// 0 .. n-1 by box_stage).  For one record the 64 lanes update 64 distinct
// cells in 64 distinct banks, so a plain read-add-write is exact.  Records are
// applied two at a time with one LDS
// round trip: both cells are read before either is written, and where the
// second record's tap lands on a cell of the first record's stencil, the lane
// adds the first record's weight for that cell, fetched from the lane that owns
// it with a cross-lane permute; the writes go out in record order, so a cell
// shared by the two ends up with both contributions.  The next pair's record
// words are read before this pair's cells are written (records never alias
// cells).  An odd last record is applied on its own.  (LDS
// float atomics measure about three times slower here, also without bank
// conflicts; groups of three or four records, or record words read eight
// records at a time, measured slower than pairs.)
__device__ inline void box_apply(GradBox &b, unsigned long long staged) {
  if (staged == 0ull) return;
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
  const int l = threadIdx.x % kWaveSize;
  const int ta = l & 3, tb = (l >> 2) & 3, tc = l >> 4;
  const int off = tc * kBoxZ + tb * kBoxY + ta;
  // tap coordinates biased by 4 in 4-bit fields: adding another record's
  // offset (x + 16 y + 256 z) leaves every field in [4, 7] exactly when the
  // shifted tap is inside that record's stencil
  const int tp = (ta + 4) + 16 * (tb + 4) + 256 * (tc + 4);
  const int l4 = 4 * l;
  const int n = __popcll(staged);
  struct Pair {
    float x[2], y[2], z[2];  // this lane's tap weights, not yet multiplied
    int cell[2], P[2], Q4[2];
  };
  // records i and i + 1 (adjacent slots)
  auto load_pair = [&](int i, Pair &q) {
    const float *r0 = b.recs + i * kRec, *r1 = r0 + kRec;
    const int4 m0 = *reinterpret_cast<const int4 *>(r0 + 12);
    const int4 m1 = *reinterpret_cast<const int4 *>(r1 + 12);
    q.x[0] = r0[ta];
    q.y[0] = r0[4 + tb];
    q.z[0] = r0[8 + tc];
    q.x[1] = r1[ta];
    q.y[1] = r1[4 + tb];
    q.z[1] = r1[8 + tc];
    q.cell[0] = m0.x + off;
    q.P[0] = m0.y;
    q.Q4[0] = m0.z;
    q.cell[1] = m1.x + off;
    q.P[1] = m1.y;
    q.Q4[1] = m1.z;
  };
  int i = 0;
  if (n >= 2) {
    Pair cur;
    load_pair(0, cur);
    for (;;) {
      const float w0 = cur.x[0] * cur.y[0] * cur.z[0];
      const float w1 = cur.x[1] * cur.y[1] * cur.z[1];
      // the first record's weight at this lane's tap of the second record
      const float c = __builtin_bit_cast(
          float, __builtin_amdgcn_ds_bpermute(l4 + cur.Q4[1] - cur.Q4[0], __builtin_bit_cast(int, w0)));
      float v0 = b.cells[cur.cell[0]];
      float v1 = b.cells[cur.cell[1]];
      const bool more = i + 3 < n;
      Pair nxt;
      if (more) load_pair(i + 2, nxt);
      const int t = tp + cur.P[1] - cur.P[0];
      v1 += (t & 0xCCC) == 0x444 ? c : 0.0f;
      b.cells[cur.cell[0]] = v0 + w0;
      b.cells[cur.cell[1]] = v1 + w1;
      i += 2;
      if (!more) break;
      cur = nxt;
    }
  }
  if (i < n) {  // an odd last record
    const float *r = b.recs + i * kRec;
    const float w = r[ta] * r[4 + tb] * r[8 + tc];
    const int cell = reinterpret_cast<const int *>(r)[12] + off;
    b.cells[cell] += w;
  }
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// The adjoint marches each ray with a group of kBwdRayGroup lanes (see
// walk_group): every lane recomputes its own samples, the group's chain gives
// each lane T_k a_k, T_{k+1} and C_{<=k} of its sample, and the lane applies
// that sample's adjoint.
#ifndef VR_BWD_RAY_GROUP
#define VR_BWD_RAY_GROUP 2
#endif
constexpr int kBwdRayGroup = VR_BWD_RAY_GROUP;
static_assert(kBwdRayGroup == 1 || kBwdRayGroup == 2 || kBwdRayGroup == 4, "ray groups lie within a quad");

template <int G, int DT>
__device__ inline void march_backward(const VolConst &v, const TfShared &s, float *sgtf, GradBox &box,
                                      const TfConst &tf, const MarchConst &mc, const Ray &r,
                                      __amdgpu_buffer_rsrc_t rs, float4 g, float4 fin, float *grad_vol) {
  const float sl2 = mc.step * 1.4426950408889634f;
  const float Tend = 1.0f - fin.w;
  // TF-gradient contributions are summed in registers for the two nodes of
  // the current TF segment (ga[0..3]: node cj, ga[4..7]: node cj + 1).  When
  // the segment moves by one node, the shared node's sums stay in registers
  // and only the node left behind is added to LDS; otherwise both are.  The
  // LDS TF gradient holds two interleaved copies, one per lane parity, so
  // the two lanes of a ray pair (usually in the same segment) do not add to
  // one address in the same instruction.
  int cj = -1;
  float ga[8] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  const int tcopy = (int)(threadIdx.x % kTfGradCopies);
  auto add_node = [&](int node, const float *val) {
    float *n0 = sgtf + 4 * node * kTfGradCopies + tcopy;
#pragma unroll
    for (int i = 0; i < 4; ++i)
      if (val[i] != 0.0f) atomicAdd(n0 + i * kTfGradCopies, val[i]);
  };
  auto flush_tf = [&]() {
    if (cj >= 0) {
      add_node(cj, ga);
      add_node(cj + 1, ga + 4);
    }
  };
  auto move_tf = [&](int j) {
    const bool up = j == cj + 1, down = j == cj - 1;
    if (cj >= 0) {
      // left behind: node cj when moving up, node cj + 1 when moving down
      float lv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) lv[i] = down ? ga[4 + i] : ga[i];
      add_node(down ? cj + 1 : cj, lv);
      if (!up && !down) add_node(cj + 1, ga + 4);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const float keep = up ? ga[4 + i] : (down ? ga[i] : 0.0f);
      ga[i] = down ? 0.0f : keep;
      ga[4 + i] = down ? keep : 0.0f;
    }
    cj = j;
  };
  bool staged = false;
  auto prep = [&](bool want, float px, float py, float pz) {
    if (grad_vol && box.cells) box_prepare(box, grad_vol, v, r, want, px, py, pz);
  };
  auto post = [&]() {
    if (grad_vol && box.cells) box_apply(box, __ballot(staged));
    staged = false;
  };
  // the taps of this lane's next lattice point are loaded while this one is
  // processed (in the adjoint every lattice point of a ray is usually visited)
  TapPrefetch<DT> pf;
  pf.ix = INT_MIN;
  float sx = 0.0f, sy = 0.0f, sz = 0.0f;  // this lane's sample: its position
  Classified cq;                          // and classification, kept for its adjoint
  auto eval = [&](int k, float px, float py, float pz) -> ChainSample {
    sx = px;
    sy = py;
    sz = pz;
    const Stencil st = make_stencil(px, py, pz);
    const float val = reconstruct_prefetched<DT>(pf, rs, v, st);
    if (k + G < r.k0 + r.ns) {
      float qx, qy, qz;
      lattice_point(r, mc.step, k + G, qx, qy, qz);
      prefetch_taps<DT>(pf, rs, v, (int)floorf(qx), (int)floorf(qy), (int)floorf(qz));
    }
    cq = classify(s, tf.K, tf.v0, tf.scale, val);
    return ChainSample{cq.c.x, cq.c.y, cq.c.z, transmit(cq.c.w, sl2)};
  };
  // TF gradient of the dsig-only adjoint of one sample with classification q
  // (its colour gradient is zero: T_k a_k = 0), n identical samples at once
  auto tf_sigma = [&](const Classified &q, float dsig, float n) {
    if (q.j != cj) move_tf(q.j);
    const float d = n * dsig;
    ga[3] = fmaf(1.0f - q.w, d, ga[3]);
    ga[7] = fmaf(q.w, d, ga[7]);
  };
  // n samples of a constant empty block (extinction 0, so a = 0 and the ray's
  // state is unchanged): only dsig is non-zero, the same for all of them
  auto flat = [&](int n, const ChainState &o, float value) {
    if (!sgtf) return;
    const Classified fq = classify(s, tf.K, tf.v0, tf.scale, value);
    float acc = g.w * Tend;
    acc = fmaf(g.x, o.T * fq.c.x - (fin.x - o.C0), acc);
    acc = fmaf(g.y, o.T * fq.c.y - (fin.y - o.C1), acc);
    acc = fmaf(g.z, o.T * fq.c.z - (fin.z - o.C2), acc);
    tf_sigma(fq, mc.step * acc, (float)n);
  };
  // adjoint of this lane's sample k, given T_k a_k, T_{k+1} and C_{<=k}
  auto take = [&](bool mine, const ChainState &o) {
    if (!mine) return;
    const float ta = o.ta, T = o.T;
    float dc0 = g.x * ta, dc1 = g.y * ta, dc2 = g.z * ta;
    float acc = g.w * Tend;
    acc = fmaf(g.x, T * cq.c.x - (fin.x - o.C0), acc);
    acc = fmaf(g.y, T * cq.c.y - (fin.y - o.C1), acc);
    acc = fmaf(g.z, T * cq.c.z - (fin.z - o.C2), acc);
    float dsig = mc.step * acc;
    if (sgtf) {
      if (cq.j != cj) move_tf(cq.j);
      float w1 = cq.w, w0 = 1.0f - cq.w;
      ga[0] = fmaf(w0, dc0, ga[0]);
      ga[1] = fmaf(w0, dc1, ga[1]);
      ga[2] = fmaf(w0, dc2, ga[2]);
      ga[3] = fmaf(w0, dsig, ga[3]);
      ga[4] = fmaf(w1, dc0, ga[4]);
      ga[5] = fmaf(w1, dc1, ga[5]);
      ga[6] = fmaf(w1, dc2, ga[6]);
      ga[7] = fmaf(w1, dsig, ga[7]);
    }
    if (grad_vol && !cq.clamped) {
      float4 a = s.node[cq.j], b = s.node[cq.j + 1];
      float dv = dc0 * (b.x - a.x);
      dv = fmaf(dc1, b.y - a.y, dv);
      dv = fmaf(dc2, b.z - a.z, dv);
      dv = fmaf(dsig, b.w - a.w, dv);
      dv *= tf.scale;
      if (dv != 0.0f) {
        const Stencil st = make_stencil(sx, sy, sz);  // (recomputed: fewer registers across the chain)
        if (box.valid)
          staged = box_stage(box, v, st, dv);
        else
          scatter_taps(grad_vol, v, st, dv);
      }
    }
  };
  float4 acc = make_float4(0.0f, 0.0f, 0.0f, 1.0f);
  walk_group<G, true>(v, s, tf, mc, r, eval, prep, take, flat, post, acc);
  if (sgtf) flush_tf();
  if (grad_vol) box_flush(box, grad_vol, v);
}

#ifdef VR_TIMELINE
__device__ unsigned long long g_timeline_bwd[kTimelineWaves * 4];
static int64_t g_timeline_bwd_records = 0;
#endif

// One wavefront item of the adjoint: wavefront w of workgroup item i.
template <int DT>
__device__ inline void backward_wave_item(const BackwardArgs &a, const TfShared &s, float *sgtf, GradBox &box,
                                          __amdgpu_buffer_rsrc_t rs, int64_t i, int w) {
#ifdef VR_TIMELINE
  const unsigned long long tl0 = __builtin_amdgcn_s_memrealtime();
#endif
  const RenderArgs &ra = a.r;
  int part;
  const SuperTile st = group_tile_of<kBwdRayGroup>(ra.order, i, ra.W, ra.H, ra.n_views, ra.chunk_edge, part);
  if (!st.valid) return;  // uniform over the wavefront
  int col, row;
  group_pixel_of<kBwdRayGroup>(st.sx, st.sy, part, w * kWaveSize + (int)(threadIdx.x % kWaveSize), col, row);
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
  march_backward<kBwdRayGroup, DT>(ra.vol, s, sgtf, box, ra.tf, ra.mc, r, rs, g, fin, a.grad_vol);
#ifdef VR_TIMELINE
  const int tx = (ra.W + kSuperEdge - 1) / kSuperEdge, ty = (ra.H + kSuperEdge - 1) / kSuperEdge;
  timeline_record(g_timeline_bwd, (size_t)i * kWavesPerWg + w, tl0, st.view * tx * ty + st.sy * tx + st.sx,
                  (threadIdx.x % kBwdRayGroup) == 0 ? (uint32_t)r.ns : 0u);
#endif
}

// LDS holds two workgroups per CU (two wavefronts per SIMD): 256 registers.
// Queued like the forward (one workgroup item per workgroup without queue
// counters); a workgroup's TF gradient stays in its LDS over all its items.
template <int DT>
__global__ __launch_bounds__(kWgSize) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_render_bwd(
    const BackwardArgs args) {
  extern __shared__ __attribute__((aligned(16))) char lds[];
  const BackwardArgs &a = kernarg<BackwardArgs>();
  const RenderArgs &ra = a.r;
  const int K = ra.tf.K;
  const uint32_t tf_bytes = tf_lds_bytes(K);
  float *sgtf = a.grad_tf ? reinterpret_cast<float *>(lds + tf_bytes) : nullptr;
  if (sgtf)
    for (int j = threadIdx.x; j < 4 * K * kTfGradCopies; j += kWgSize) sgtf[j] = 0.0f;
  GradBox box;
  box.valid = false;
  box.ox = box.oy = box.oz = 0;
  box.cells = nullptr;
  if (a.grad_vol && a.use_box) {
    float *boxes = reinterpret_cast<float *>(lds + box_lds_offset(K, a.grad_tf != nullptr));
    const int wave = threadIdx.x / kWaveSize;
    box.cells = boxes + wave * (kBoxCells + kWaveSize * kRec);
    box.recs = box.cells + kBoxCells;
    for (int i = threadIdx.x % kWaveSize; i < kBoxCells; i += kWaveSize) box.cells[i] = 0.0f;
  }
  TfShared s = carve_tf(lds, K);
  const bool tf_ok = load_tf(s, ra.tf);  // ends with a barrier, which also orders the zeroing
  if (!tf_ok) {
    // uniform over the launch: every workgroup fills its share of the
    // gradients with NaN and nothing is accumulated
    const float q = __builtin_nanf("");
    const int64_t nvox = (int64_t)ra.vol.nx * ra.vol.ny * ra.vol.nz;
    if (a.grad_vol)
      for (int64_t i = (int64_t)blockIdx.x * kWgSize + threadIdx.x; i < nvox; i += (int64_t)gridDim.x * kWgSize)
        a.grad_vol[i] = q;
    if (a.grad_tf && blockIdx.x == 0)
      for (int j = threadIdx.x; j < 4 * K; j += kWgSize) a.grad_tf[j] = q;
    return;
  }
  __amdgpu_buffer_rsrc_t rs = make_rsrc(ra.vol.data, ra.vol.bytes);
  if (!ra.queue) {
    int part;
    if (!group_tile_of<kBwdRayGroup>(ra.order, blockIdx.x, ra.W, ra.H, ra.n_views, ra.chunk_edge, part).valid)
      return;  // uniform over the workgroup
    backward_wave_item<DT>(a, s, sgtf, box, rs, blockIdx.x, (int)(threadIdx.x / kWaveSize));
  } else {
    const int x = (int)(blockIdx.x % kXcds);
    int w = 0;
    int64_t i = 0;
    while (next_wave_item(ra.queue, (uint32_t)ra.queue_items, x, i, w))
      backward_wave_item<DT>(a, s, sgtf, box, rs, i, w);
  }
  if (sgtf) {
    __syncthreads();
    for (int j = threadIdx.x; j < 4 * K; j += kWgSize) {
      float val = 0.0f;
#pragma unroll
      for (int c = 0; c < kTfGradCopies; ++c) val += sgtf[j * kTfGradCopies + c];
      if (val != 0.0f) unsafeAtomicAdd(a.grad_tf + j, val);
    }
  }
}

hipError_t launch_render_backward(const BackwardArgs &a0, hipStream_t s) {
  BackwardArgs a = a0;
  const RenderArgs &ra = a.r;
  int64_t grid = group_grid(render_grid(ra), kBwdRayGroup);
#ifdef VR_TIMELINE
  g_timeline_bwd_records = grid * (kWgSize / kWaveSize);
#endif
  uint32_t lds = tf_lds_bytes(ra.tf.K) + (a.grad_tf ? (uint32_t)ra.tf.K * 16u * kTfGradCopies : 0u);
  const uint32_t box_bytes = (uint32_t)(kWgSize / kWaveSize) * (kBoxCells + kWaveSize * kRec) * 4u;
  const uint32_t with_box = box_lds_offset(ra.tf.K, a.grad_tf != nullptr) + box_bytes;
  a.use_box = (a.grad_vol && with_box <= max_lds_per_workgroup()) ? 1 : 0;
  if (a.use_box) lds = with_box;
  const void *fn = nullptr;
  switch (ra.vol.dtype) {
  case kU16: fn = reinterpret_cast<const void *>(&k_render_bwd<kU16>); break;
  case kI16: fn = reinterpret_cast<const void *>(&k_render_bwd<kI16>); break;
  case kF32: fn = reinterpret_cast<const void *>(&k_render_bwd<kF32>); break;
  default: return hipErrorInvalidValue;
  }
  hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  a.r.queue = nullptr;
  a.r.queue_items = 0;
  if (ra.order) {
    const int64_t resident = resident_workgroups(fn, lds);
    if (resident >= kXcds && resident < grid) {
      a.r.queue = reinterpret_cast<uint32_t *>(const_cast<int32_t *>(ra.order) + tile_order_count(ra));
      a.r.queue_items = (int32_t)(grid / kXcds * kWavesPerWg);
      grid = resident;
    }
  }
  switch (ra.vol.dtype) {
  case kU16: hipLaunchKernelGGL(k_render_bwd<kU16>, dim3((unsigned)grid), dim3(kWgSize), lds, s, a); break;
  case kI16: hipLaunchKernelGGL(k_render_bwd<kI16>, dim3((unsigned)grid), dim3(kWgSize), lds, s, a); break;
  default: hipLaunchKernelGGL(k_render_bwd<kF32>, dim3((unsigned)grid), dim3(kWgSize), lds, s, a); break;
  }
  return hipGetLastError();
}

#ifdef VR_TIMELINE
int64_t timeline_copy_bwd(unsigned long long *host, int64_t max) {
  const int64_t n = std::min<int64_t>(std::min<int64_t>(g_timeline_bwd_records, kTimelineWaves), max);
  if (hipDeviceSynchronize() != hipSuccess) return -1;
  if (n > 0 && hipMemcpyFromSymbol(host, HIP_SYMBOL(g_timeline_bwd), (size_t)n * 4 * sizeof(unsigned long long)) != hipSuccess)
    return -1;
  return g_timeline_bwd_records;
}
#endif

}  // namespace vr
