// api.cpp -- the C ABI of include/vr.h (except serving, in serve.cpp):
// argument validation, FP64 camera constants, launch configuration and
// error reporting.  Kernels live in the .hip files.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdarg>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "vr.h"
#include "vr_internal.h"
#include "vr_timeline.h"

struct vr_blocks {
  const void *data;
  int32_t dtype;
  int64_t nx, ny, nz;
  int32_t edge;
  int32_t nbx, nby, nbz;
  float2 *minmax;
  float2 *minmax_cr;  // ranges widened for Catmull-Rom samples
  int device;
};

struct vr_preint {
  float4 *table;  // K x K (C_r, C_g, C_b, alpha), entry (i, j) at i K + j
  int32_t K;
  float step, v0, v1;
  const float *tf_table;  // the TF it was built from (checked at render)
};

namespace vr {

static thread_local std::string g_last_error;

vr_status fail(vr_status s, const char *fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

vr_status hip_fail(hipError_t e, const char *what) {
  return fail(VR_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

static bool finite3(const double v[3]) { return std::isfinite(v[0]) && std::isfinite(v[1]) && std::isfinite(v[2]); }

vr_status check_volume(const vr_volume *v, VolConst *out) {
  if (!v) return fail(VR_E_INVALID_ARG, "volume is NULL");
  if (!v->data) return fail(VR_E_INVALID_ARG, "volume data is NULL");
  if (v->dtype != VR_U16 && v->dtype != VR_I16 && v->dtype != VR_F32)
    return fail(VR_E_INVALID_ARG, "unknown volume dtype %d", v->dtype);
  if (v->nx <= 0 || v->ny <= 0 || v->nz <= 0)
    return fail(VR_E_INVALID_ARG, "volume dims must be positive (%lld, %lld, %lld)", (long long)v->nx,
                (long long)v->ny, (long long)v->nz);
  if ((reinterpret_cast<uintptr_t>(v->data) & 3u) != 0)
    return fail(VR_E_INVALID_ARG, "volume data must be 4-byte aligned");
  const int64_t esz = v->dtype == VR_F32 ? 4 : 2;
  const double bytes = (double)v->nx * (double)v->ny * (double)v->nz * (double)esz;
  if (v->nx > (1 << 20) || v->ny > (1 << 20) || v->nz > (1 << 20) || bytes >= 4294967296.0)
    return fail(VR_E_UNSUPPORTED, "volume of %.0f bytes exceeds the 4 GiB per-volume limit", bytes);
  if (out) {
    out->data = v->data;
    out->dtype = v->dtype;
    out->nx = (int32_t)v->nx;
    out->ny = (int32_t)v->ny;
    out->nz = (int32_t)v->nz;
    out->bytes = (uint32_t)bytes;
    out->minmax = nullptr;
    out->nbx = out->nby = out->nbz = 0;
    out->edge = 0;
    out->edge_shift = 0;
    out->row_even = (v->nx % 2) == 0 ? 1 : 0;
  }
  return VR_OK;
}

vr_status check_tf_fields(const void *table, int32_t K, float v0, float v1, TfConst *out) {
  if (!table) return fail(VR_E_INVALID_ARG, "TF table is NULL");
  if (K < 2 || K > VR_MAX_TF_NODES) return fail(VR_E_INVALID_ARG, "TF node count K=%d outside [2, %d]", K, VR_MAX_TF_NODES);
  if (!std::isfinite(v0) || !std::isfinite(v1) || !(v1 > v0))
    return fail(VR_E_INVALID_ARG, "TF value range must be finite with v1 > v0 (%g, %g)", (double)v0, (double)v1);
  if ((reinterpret_cast<uintptr_t>(table) & 15u) != 0) return fail(VR_E_INVALID_ARG, "TF table must be 16-byte aligned");
  if (out) {
    out->table = static_cast<const float *>(table);
    out->K = K;
    out->v0 = v0;
    out->scale = (float)(K - 1) / (v1 - v0);
    out->status = tf_status_word();
  }
  return VR_OK;
}

vr_status check_camera(const vr_camera *c, CamConst *out) {
  if (!c) return fail(VR_E_INVALID_ARG, "camera is NULL");
  if (c->width <= 0 || c->height <= 0 || c->width > 32768 || c->height > 32768)
    return fail(VR_E_INVALID_ARG, "image size %dx%d outside [1, 32768]", c->width, c->height);
  if (c->projection != 0 && c->projection != 1) return fail(VR_E_INVALID_ARG, "projection must be 0 or 1");
  if (!finite3(c->eye) || !finite3(c->right) || !finite3(c->up) || !finite3(c->forward))
    return fail(VR_E_INVALID_ARG, "camera vectors must be finite");
  const double fn = c->forward[0] * c->forward[0] + c->forward[1] * c->forward[1] + c->forward[2] * c->forward[2];
  if (!(fn > 0.0)) return fail(VR_E_INVALID_ARG, "camera forward vector is zero");
  if (c->projection == 1) {
    if (!std::isfinite(c->fov_y) || !(c->fov_y > 0.0) || !(c->fov_y < M_PI))
      return fail(VR_E_INVALID_ARG, "fov_y must be in (0, pi)");
  } else {
    if (!std::isfinite(c->ortho_w) || !std::isfinite(c->ortho_h) || !(c->ortho_w > 0.0) || !(c->ortho_h > 0.0))
      return fail(VR_E_INVALID_ARG, "ortho extents must be positive");
  }
  if (out) {
    for (int k = 0; k < 3; ++k) {
      out->eye[k] = c->eye[k];
      out->right[k] = c->right[k];
      out->up[k] = c->up[k];
      out->fwd[k] = c->forward[k];
    }
    out->th = c->projection == 1 ? std::tan(0.5 * c->fov_y) : 0.0;
    out->hw = 0.5 * c->ortho_w;
    out->hh = 0.5 * c->ortho_h;
    out->proj = c->projection;
    out->W = c->width;
    out->H = c->height;
    out->pad = 0;
  }
  return VR_OK;
}

vr_status check_march(float step, float ert, int32_t use_skip, MarchConst *out) {
  if (!std::isfinite(step) || !(step >= 1.0f / 1024.0f) || !(step <= 1024.0f))
    return fail(VR_E_INVALID_ARG, "step must be finite and within [1/1024, 1024] voxels (got %g)", (double)step);
  if (out) {
    out->step = step;
    out->ert = (ert > 0.0f && ert < 1.0f) ? ert : 0.0f;
    out->skip = use_skip ? 1 : 0;
    out->flat = 0;
  }
  return VR_OK;
}

vr_status check_shading(const vr_shading *sh, ShadeConst *out) {
  if (!sh) return fail(VR_E_INVALID_ARG, "shading is NULL");
  const float k[3] = {sh->ambient, sh->diffuse, sh->specular};
  for (float x : k)
    if (!std::isfinite(x) || x < 0.0f) return fail(VR_E_INVALID_ARG, "ambient/diffuse/specular must be finite and >= 0");
  if (!std::isfinite(sh->shininess) || !(sh->shininess >= 1.0f) || !(sh->shininess <= 1024.0f))
    return fail(VR_E_INVALID_ARG, "shininess must be within [1, 1024] (got %g)", (double)sh->shininess);
  if (!std::isfinite(sh->grad_min) || !(sh->grad_min > 0.0f))
    return fail(VR_E_INVALID_ARG, "grad_min must be finite and > 0");
  double L[3] = {0.0, 0.0, 0.0};
  if (!sh->headlight) {
    double n = 0.0;
    for (int a = 0; a < 3; ++a) {
      if (!std::isfinite(sh->light[a])) return fail(VR_E_INVALID_ARG, "light direction is not finite");
      n += (double)sh->light[a] * (double)sh->light[a];
    }
    if (!(n > 1e-30)) return fail(VR_E_INVALID_ARG, "light direction has zero length");
    n = std::sqrt(n);
    for (int a = 0; a < 3; ++a) L[a] = (double)sh->light[a] / n;
  }
  if (out) {
    out->ka = sh->ambient;
    out->kd = sh->diffuse;
    out->ks = sh->specular;
    out->shininess = sh->shininess;
    for (int a = 0; a < 3; ++a) out->light[a] = (float)L[a];
    out->headlight = sh->headlight ? 1 : 0;
    out->grad_min = sh->grad_min;
    out->pad = 0;
  }
  return VR_OK;
}

vr_status attach_blocks(const vr_blocks *b, const vr_volume *v, VolConst *vc) {
  if (!b) return fail(VR_E_INVALID_ARG, "use_skip needs blocks");
  if (b->data != v->data || b->dtype != v->dtype || b->nx != v->nx || b->ny != v->ny || b->nz != v->nz)
    return fail(VR_E_INVALID_ARG, "blocks were built for another volume");
  vc->minmax = b->minmax;
  vc->nbx = b->nbx;
  vc->nby = b->nby;
  vc->nbz = b->nbz;
  vc->edge = b->edge;
  vc->edge_shift = __builtin_ctz((unsigned)b->edge);
  return VR_OK;
}

uint32_t max_lds_per_workgroup() {
  int dev = 0, v = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 65536u;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
    return 65536u;
  return (uint32_t)v;
}

int32_t chunk_edge_setting() {
  static const int32_t ce = [] {
    const char *e = std::getenv("VR_CHUNK_EDGE");
    int v = e ? std::atoi(e) : kDefaultChunkEdge;
    return (v == 1 || v == 2 || v == 4 || v == 8) ? v : kDefaultChunkEdge;
  }();
  return ce;
}

// Validate the common arguments of vr_render / vr_render_backward and fill
// the launch arguments (cameras excluded).
vr_status prepare_render(const vr_volume *vol, const vr_blocks *blocks, const vr_camera *cams, int32_t n_cams,
                         const vr_tf *tf, const vr_params *p, RenderArgs *a) {
  memset(a, 0, sizeof(*a));
  vr_status s = check_volume(vol, &a->vol);
  if (s) return s;
  if (!tf) return fail(VR_E_INVALID_ARG, "tf is NULL");
  if ((s = check_tf_fields(tf->table, tf->K, tf->v0, tf->v1, &a->tf))) return s;
  if (!p) return fail(VR_E_INVALID_ARG, "params is NULL");
  if ((s = check_march(p->step, p->ert_threshold, p->use_skip, &a->mc))) return s;
  if (!cams || n_cams <= 0) return fail(VR_E_INVALID_ARG, "need at least one camera");
  for (int32_t i = 0; i < n_cams; ++i) {
    if ((s = check_camera(&cams[i], nullptr))) return s;
    if (cams[i].width != cams[0].width || cams[i].height != cams[0].height)
      return fail(VR_E_INVALID_ARG, "all cameras must share one image size");
  }
  if (p->filter != VR_FILTER_BSPLINE && p->filter != VR_FILTER_CATMULL_ROM &&
      p->filter != VR_FILTER_BSPLINE_PRECLASSIFIED && p->filter != VR_FILTER_TRILINEAR)
    return fail(VR_E_INVALID_ARG, "unknown filter %d", p->filter);
  if (p->use_skip && (s = attach_blocks(blocks, vol, &a->vol))) return s;
  a->filter = p->filter;
  if (p->use_skip && p->filter == VR_FILTER_CATMULL_ROM) a->vol.minmax = blocks->minmax_cr;
  a->counters = reinterpret_cast<unsigned long long *>(p->counters);
  a->W = cams[0].width;
  a->H = cams[0].height;
  a->chunk_edge = chunk_edge_setting();
  return VR_OK;
}

}  // namespace vr

using namespace vr;

extern "C" {

const char *vr_last_error(void) { return g_last_error.c_str(); }

int vr_abi_version(void) { return VR_ABI_VERSION; }

vr_status vr_build_blocks(const vr_volume *vol, int32_t block_edge, void *stream, vr_blocks **out) {
  if (!out) return fail(VR_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  VolConst vc;
  vr_status s = check_volume(vol, &vc);
  if (s) return s;
  if (block_edge < 4 || block_edge > 64 || (block_edge & (block_edge - 1)) != 0)
    return fail(VR_E_INVALID_ARG, "block edge %d is not a power of two in [4, 64]", block_edge);
  vr_blocks *b = new (std::nothrow) vr_blocks();
  if (!b) return fail(VR_E_OOM, "host allocation failed");
  b->data = vol->data;
  b->dtype = vol->dtype;
  b->nx = vol->nx;
  b->ny = vol->ny;
  b->nz = vol->nz;
  b->edge = block_edge;
  b->nbx = (int32_t)((vol->nx + block_edge - 1) / block_edge);
  b->nby = (int32_t)((vol->ny + block_edge - 1) / block_edge);
  b->nbz = (int32_t)((vol->nz + block_edge - 1) / block_edge);
  (void)hipGetDevice(&b->device);
  const size_t nb = (size_t)b->nbx * b->nby * b->nbz;
  hipError_t e = hipMalloc(&b->minmax, 2 * nb * sizeof(float2));
  if (e != hipSuccess) {
    delete b;
    return fail(VR_E_OOM, "hipMalloc of %zu block bytes: %s", 2 * nb * sizeof(float2), hipGetErrorString(e));
  }
  b->minmax_cr = b->minmax + nb;
  vc.nbx = b->nbx;
  vc.nby = b->nby;
  vc.nbz = b->nbz;
  vc.edge = block_edge;
  vc.edge_shift = __builtin_ctz((unsigned)block_edge);
  e = launch_block_minmax(vc, b->minmax, (hipStream_t)stream);
  if (e == hipSuccess) e = launch_widen_minmax(b->minmax, b->minmax_cr, (int64_t)nb, kCatmullRomWiden, (hipStream_t)stream);
  if (e != hipSuccess) {
    (void)hipFree(b->minmax);
    delete b;
    return hip_fail(e, "block min/max launch");
  }
  *out = b;
  return VR_OK;
}

vr_status vr_blocks_info(const vr_blocks *b, int64_t dims_out[3], int32_t *edge_out) {
  if (!b) return fail(VR_E_INVALID_ARG, "blocks is NULL");
  if (dims_out) {
    dims_out[0] = b->nbx;
    dims_out[1] = b->nby;
    dims_out[2] = b->nbz;
  }
  if (edge_out) *edge_out = b->edge;
  return VR_OK;
}

vr_status vr_blocks_minmax(const vr_blocks *b, float *dst, int64_t dst_count, void *stream) {
  if (!b || !dst) return fail(VR_E_INVALID_ARG, "blocks or destination is NULL");
  const int64_t nb = (int64_t)b->nbx * b->nby * b->nbz;
  if (dst_count < 2 * nb) return fail(VR_E_INVALID_ARG, "destination holds %lld floats, need %lld", (long long)dst_count, (long long)(2 * nb));
  hipError_t e = hipMemcpyAsync(dst, b->minmax, (size_t)nb * sizeof(float2), hipMemcpyDeviceToDevice, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "copy block min/max");
  return VR_OK;
}

vr_status vr_block_occupancy(const vr_blocks *b, const vr_tf *tf, uint8_t *occ, int64_t n, void *stream) {
  if (!b || !tf || !occ) return fail(VR_E_INVALID_ARG, "blocks, tf or destination is NULL");
  const int64_t nb = (int64_t)b->nbx * b->nby * b->nbz;
  if (n < nb) return fail(VR_E_INVALID_ARG, "destination holds %lld bytes, need %lld", (long long)n, (long long)nb);
  TfConst tc;
  vr_status s = check_tf_fields(tf->table, tf->K, tf->v0, tf->v1, &tc);
  if (s) return s;
  VolConst vc;
  memset(&vc, 0, sizeof(vc));
  vc.minmax = b->minmax;
  vc.nbx = b->nbx;
  vc.nby = b->nby;
  vc.nbz = b->nbz;
  vc.edge = b->edge;
  vc.edge_shift = __builtin_ctz((unsigned)b->edge);
  hipError_t e = launch_block_occupancy(vc, tc, occ, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "block occupancy launch");
  return VR_OK;
}

void vr_blocks_free(vr_blocks *b) {
  if (!b) return;
  (void)hipFree(b->minmax);
  delete b;
}

}  // extern "C"

namespace vr {

// Calls that could not allocate or build their per-call occupancy bits or
// workgroup order and rendered with the slower paths (same result).
std::atomic<uint64_t> g_fallback_occupancy{0}, g_fallback_order{0};

vr_status render_views(RenderArgs &a, const vr_camera *cams, int32_t n_cams, float *out_rgba, void *stream,
                       const float4 *preint, const RenderScratch *scratch) {
  const size_t view_floats = (size_t)a.W * a.H * 4;
  hipStream_t st = (hipStream_t)stream;
  // the blocks' occupancy under this TF, once for all views (without it the
  // kernels decide from min/max and the TF on every block change)
  uint32_t *bits = nullptr;
  bool own_bits = false, radius = false;
  if (a.mc.skip && a.vol.minmax) {
    if (scratch) {
      bits = scratch->occ;
    } else if (hipMallocAsync(reinterpret_cast<void **>(&bits), occupancy_bytes(a.vol), st) != hipSuccess) {
      (void)hipGetLastError();
      bits = nullptr;
    } else {
      own_bits = true;
    }
    if (!bits) g_fallback_occupancy.fetch_add(1, std::memory_order_relaxed);
    if (bits) {
      // (pre-integration leaps block by block: its cells span two blocks)
      if (!preint && occupancy_planes_fit(a.vol, a.tf.K)) {
        radius = launch_occupancy_planes(a.vol, a.tf, bits, st) == hipSuccess;
        if (!radius) (void)hipGetLastError();
      }
      if (!radius && launch_occupancy_bits(a.vol, a.tf, bits, st) != hipSuccess) {
        (void)hipGetLastError();
        if (own_bits) (void)hipFreeAsync(bits, st);
        bits = nullptr;
        own_bits = false;
        g_fallback_occupancy.fetch_add(1, std::memory_order_relaxed);
      }
    }
  }
  a.vol.occ = bits;
  a.vol.occ_radius = radius ? kEmptyRadiusMax : 0;
  // views per launch: what the kernel arguments carry and, with scratch,
  // what its order area holds
  int32_t per_launch = kMaxCamsPerLaunch;
  if (scratch) {
    const int64_t tiles = (int64_t)((a.W + kSuperEdge - 1) / kSuperEdge) * ((a.H + kSuperEdge - 1) / kSuperEdge);
    per_launch = (int32_t)std::min<int64_t>(kMaxCamsPerLaunch, (scratch->order_ints - kOrderQueueInts) / tiles);
  }
  vr_status result = VR_OK;
  for (int32_t v0 = 0; v0 < n_cams; v0 += per_launch) {
    const int32_t n = std::min(per_launch, n_cams - v0);
    for (int32_t i = 0; i < n; ++i) check_camera(&cams[v0 + i], &a.cams[i]);
    a.n_views = n;
    a.out = out_rgba + (size_t)v0 * view_floats;
    bool own_order = false;
    if (scratch) {
      a.order = launch_tile_order(a, scratch->order, st) == hipSuccess ? scratch->order : nullptr;
      if (!a.order) (void)hipGetLastError();
    } else {
      a.order = make_tile_order(a, st);
      own_order = a.order != nullptr;
    }
    if (!a.order) g_fallback_order.fetch_add(1, std::memory_order_relaxed);
    hipError_t e = preint ? launch_render_preint(a, preint, st) : launch_render(a, st);
    if (own_order) (void)hipFreeAsync(const_cast<int32_t *>(a.order), st);
    a.order = nullptr;
    if (e != hipSuccess) {
      result = hip_fail(e, "render launch");
      break;
    }
  }
  if (own_bits) (void)hipFreeAsync(bits, st);
  a.vol.occ = nullptr;
  a.vol.occ_radius = 0;
  return result;
}

}  // namespace vr

extern "C" {

vr_status vr_render(const vr_volume *vol, const vr_blocks *blocks, const vr_camera *cams, int32_t n_cams,
                    const vr_tf *tf, const vr_params *p, float *out_rgba, void *stream) {
  RenderArgs a;
  vr_status s = prepare_render(vol, blocks, cams, n_cams, tf, p, &a);
  if (s) return s;
  if (!out_rgba) return fail(VR_E_INVALID_ARG, "out_rgba is NULL");
  return render_views(a, cams, n_cams, out_rgba, stream, nullptr, nullptr);
}

vr_status vr_render_shaded(const vr_volume *vol, const vr_blocks *blocks, const vr_camera *cams, int32_t n_cams,
                           const vr_tf *tf, const vr_params *p, const vr_shading *shading, float *out_rgba,
                           void *stream) {
  RenderArgs a;
  vr_status s = prepare_render(vol, blocks, cams, n_cams, tf, p, &a);
  if (s) return s;
  if (p->filter != VR_FILTER_BSPLINE) return fail(VR_E_UNSUPPORTED, "local lighting uses the cubic B-spline only");
  if ((s = check_shading(shading, &a.shade))) return s;
  if (!out_rgba) return fail(VR_E_INVALID_ARG, "out_rgba is NULL");
  a.shaded = 1;
  return render_views(a, cams, n_cams, out_rgba, stream, nullptr, nullptr);
}

vr_status vr_preint_build(const vr_tf *tf, float step, void *stream, vr_preint **out) {
  if (!out) return fail(VR_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!tf) return fail(VR_E_INVALID_ARG, "tf is NULL");
  TfConst tc;
  vr_status s = check_tf_fields(tf->table, tf->K, tf->v0, tf->v1, &tc);
  if (s) return s;
  MarchConst mc;
  if ((s = check_march(step, 0.0f, 0, &mc))) return s;
  vr_preint *t = new (std::nothrow) vr_preint();
  if (!t) return fail(VR_E_OOM, "host allocation failed");
  t->K = tf->K;
  t->step = step;
  t->v0 = tf->v0;
  t->v1 = tf->v1;
  t->tf_table = tf->table;
  const size_t bytes = (size_t)tf->K * tf->K * sizeof(float4);
  hipError_t e = hipMalloc(&t->table, bytes);
  if (e != hipSuccess) {
    delete t;
    return fail(VR_E_OOM, "hipMalloc of %zu table bytes: %s", bytes, hipGetErrorString(e));
  }
  e = launch_preint_table(tf->table, tf->K, step, t->table, tc.status, (hipStream_t)stream);
  if (e != hipSuccess) {
    (void)hipFree(t->table);
    delete t;
    return hip_fail(e, "pre-integration table launch");
  }
  *out = t;
  return VR_OK;
}

vr_status vr_preint_table(const vr_preint *t, float *dst, int64_t dst_count, void *stream) {
  if (!t || !dst) return fail(VR_E_INVALID_ARG, "table or destination is NULL");
  const int64_t n = (int64_t)t->K * t->K * 4;
  if (dst_count < n) return fail(VR_E_INVALID_ARG, "destination holds %lld floats, need %lld", (long long)dst_count, (long long)n);
  hipError_t e = hipMemcpyAsync(dst, t->table, (size_t)n * sizeof(float), hipMemcpyDeviceToDevice, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "copy pre-integration table");
  return VR_OK;
}

void vr_preint_free(vr_preint *t) {
  if (!t) return;
  (void)hipFree(t->table);
  delete t;
}

vr_status vr_render_preint(const vr_volume *vol, const vr_blocks *blocks, const vr_camera *cams, int32_t n_cams,
                           const vr_tf *tf, const vr_params *p, const vr_preint *table, float *out_rgba,
                           void *stream) {
  RenderArgs a;
  vr_status s = prepare_render(vol, blocks, cams, n_cams, tf, p, &a);
  if (s) return s;
  if (p->filter != VR_FILTER_BSPLINE) return fail(VR_E_UNSUPPORTED, "pre-integration uses the cubic B-spline only");
  if (!table) return fail(VR_E_INVALID_ARG, "pre-integration table is NULL");
  if (table->K != tf->K || table->v0 != tf->v0 || table->v1 != tf->v1 || table->tf_table != tf->table ||
      table->step != p->step)
    return fail(VR_E_INVALID_ARG, "the pre-integration table was built for another TF or step");
  if (!out_rgba) return fail(VR_E_INVALID_ARG, "out_rgba is NULL");
  return render_views(a, cams, n_cams, out_rgba, stream, table->table, nullptr);
}

vr_status vr_prefilter_bspline(const vr_volume *vol, float *coeff_out, void *stream) {
  VolConst vc;
  vr_status s = check_volume(vol, &vc);
  if (s) return s;
  if (!coeff_out) return fail(VR_E_INVALID_ARG, "coeff_out is NULL");
  // pivots of tridiag(1, 4, 1) with end diagonals 5, per axis length (FP64,
  // rounded once); the table travels with the launch in a small device buffer
  const int64_t dims[3] = {vol->nx, vol->ny, vol->nz};
  std::vector<float> coef;
  for (int a = 0; a < 3; ++a) {
    const int64_t n = dims[a];
    std::vector<double> piv((size_t)n), sup((size_t)n, 0.0);
    for (int64_t i = 0; i < n; ++i) {
      const double diag = (i == 0 || i == n - 1) ? 5.0 : 4.0;
      piv[(size_t)i] = i == 0 ? diag : diag - sup[(size_t)i - 1];
      sup[(size_t)i] = i < n - 1 ? 1.0 / piv[(size_t)i] : 0.0;
    }
    for (int64_t i = 0; i < n; ++i) coef.push_back((float)(1.0 / piv[(size_t)i]));
    for (int64_t i = 0; i < n; ++i) coef.push_back((float)sup[(size_t)i]);
  }
  float *dcoef = nullptr;
  hipError_t e = hipMallocAsync((void **)&dcoef, coef.size() * sizeof(float), (hipStream_t)stream);
  if (e != hipSuccess) return fail(VR_E_OOM, "prefilter table allocation: %s", hipGetErrorString(e));
  if ((e = hipMemcpyAsync(dcoef, coef.data(), coef.size() * sizeof(float), hipMemcpyHostToDevice,
                          (hipStream_t)stream)) != hipSuccess ||
      (e = hipStreamSynchronize((hipStream_t)stream)) != hipSuccess) {
    (void)hipFreeAsync(dcoef, (hipStream_t)stream);
    return hip_fail(e, "prefilter table upload");
  }
  e = launch_prefilter(vc, coeff_out, dcoef, (hipStream_t)stream);
  (void)hipFreeAsync(dcoef, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "prefilter launch");
  return VR_OK;
}

vr_status vr_fallback_counts(uint64_t *occupancy, uint64_t *order) {
  if (!occupancy || !order) return fail(VR_E_INVALID_ARG, "occupancy and order are required");
  *occupancy = g_fallback_occupancy.load(std::memory_order_relaxed);
  *order = g_fallback_order.load(std::memory_order_relaxed);
  return VR_OK;
}

vr_status vr_timeline_read(int32_t kernel, uint64_t *host_out, uint64_t max_records, uint64_t *n_records) {
#ifdef VR_TIMELINE
  if (kernel != VR_TIMELINE_FORWARD && kernel != VR_TIMELINE_ADJOINT)
    return fail(VR_E_INVALID_ARG, "unknown timeline kernel %d", kernel);
  if (!host_out || !n_records) return fail(VR_E_INVALID_ARG, "host_out and n_records are required");
  const int64_t max = (int64_t)std::min<uint64_t>(max_records, (uint64_t)kTimelineWaves);
  unsigned long long *h = reinterpret_cast<unsigned long long *>(host_out);
  const int64_t n = kernel == VR_TIMELINE_FORWARD ? timeline_copy_fwd(h, max) : timeline_copy_bwd(h, max);
  if (n < 0) return fail(VR_E_DEVICE, "timeline copy failed");
  *n_records = (uint64_t)n;
  return VR_OK;
#else
  (void)kernel;
  (void)host_out;
  (void)max_records;
  (void)n_records;
  return fail(VR_E_UNSUPPORTED, "this library keeps no timeline (built without VR_TIMELINE)");
#endif
}

vr_status vr_render_backward(const vr_volume *vol, const vr_blocks *blocks, const vr_camera *cams, int32_t n_cams,
                             const vr_tf *tf, const vr_params *p, const float *out_rgba, const float *grad_rgba,
                             float *grad_volume, float *grad_tf, void *stream) {
  BackwardArgs b;
  vr_status s = prepare_render(vol, blocks, cams, n_cams, tf, p, &b.r);
  if (s) return s;
  if (p->filter != VR_FILTER_BSPLINE) return fail(VR_E_UNSUPPORTED, "the adjoint is of the cubic B-spline render");
  if (!out_rgba || !grad_rgba) return fail(VR_E_INVALID_ARG, "out_rgba and grad_rgba are required");
  if (!p->use_skip && blocks && (s = attach_blocks(blocks, vol, &b.r.vol))) return s;
  if (grad_tf) b.r.mc.skip = 0;  // zero-extinction nodes still receive TF gradients
  // every sample is visited: with the blocks' min/max, samples in constant
  // empty blocks take the constant without reconstruction
  b.r.mc.flat = !b.r.mc.skip && b.r.vol.minmax ? 1 : 0;
  b.r.counters = nullptr;
  hipStream_t st = (hipStream_t)stream;
  const int64_t nvox = (int64_t)vol->nx * vol->ny * vol->nz;
  hipError_t e;
  if (grad_volume && (e = launch_fill_zero(grad_volume, nvox, st)) != hipSuccess) return hip_fail(e, "zero grad_volume");
  if (grad_tf && (e = launch_fill_zero(grad_tf, (int64_t)tf->K * 4, st)) != hipSuccess) return hip_fail(e, "zero grad_tf");
  if (!grad_volume && !grad_tf) return VR_OK;
  const size_t view_floats = (size_t)b.r.W * b.r.H * 4;
  for (int32_t v0 = 0; v0 < n_cams; v0 += kMaxCamsPerLaunch) {
    const int32_t n = std::min(kMaxCamsPerLaunch, n_cams - v0);
    for (int32_t i = 0; i < n; ++i) check_camera(&cams[v0 + i], &b.r.cams[i]);
    b.r.n_views = n;
    b.r.out = nullptr;
    b.out_rgba = out_rgba + (size_t)v0 * view_floats;
    b.grad_rgba = grad_rgba + (size_t)v0 * view_floats;
    b.grad_vol = grad_volume;
    b.grad_tf = grad_tf;
    b.use_box = 0;
    b.pad = 0;
    b.r.order = make_tile_order(b.r, st);
    if (!b.r.order) g_fallback_order.fetch_add(1, std::memory_order_relaxed);
    e = launch_render_backward(b, st);
    if (b.r.order) (void)hipFreeAsync(const_cast<int32_t *>(b.r.order), st);
    b.r.order = nullptr;
    if (e != hipSuccess) return hip_fail(e, "backward launch");
  }
  return VR_OK;
}

}  // extern "C"
