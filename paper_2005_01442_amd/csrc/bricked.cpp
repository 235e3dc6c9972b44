// bricked.cpp -- out-of-core volumes: host-resident bricks, a device brick
// pool with a page table, and front-to-back rendering passes.
//
// The paper's block decomposition renders volumes that do not fit GPU memory
// one block at a time (Section 2: blocks overlapping by the voxels a cubic
// stencil reads, smaller blocks at the far faces, completely empty blocks
// excluded; Fig. 3 and the pros and cons that follow).  A brick here is a
// block's footprint, copied once into pinned host memory.  Rendering a view:
//   1. TF occupancy of every brick (the blocks' min/max test, on the device);
//   2. the occupied bricks in a front-to-back order for the camera: along
//      each axis a ray moves away from the eye's slab, so the sum over the
//      axes of |brick index - eye slab index| grows at every brick a ray
//      enters (orthographic: the sum of sign(d_a) * index); sorting by it
//      orders the bricks of every ray;
//   3. passes over consecutive runs of that order, as many bricks as the pool
//      holds: bricks already resident stay, missing ones are copied in, the
//      page table lists the pass's bricks, and the pass kernel continues every
//      ray through them from the state earlier passes left;
//   4. the RGBA image from the final state.
// Empty bricks are never copied; their samples add exactly zero.
#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <new>
#include <thread>
#include <vector>

#include "vr_internal.h"

namespace vr {
// Device memory bricks of several volumes take turns in (a server's shared
// pool): the volume that renders owns all of it; a volume that renders after
// another finds none of its bricks resident.
struct BrickArena {
  char *mem = nullptr;
  uint64_t bytes = 0;
  const vr_bricked *owner = nullptr;
};
}  // namespace vr

struct vr_bricked {
  vr::BrickArena *arena;   // shared pool (nullptr: the pool below is this volume's own)
  int32_t dtype;
  int64_t nx, ny, nz;
  int32_t E, S;
  int32_t nbx, nby, nbz;
  int64_t nbricks;
  int64_t esz;
  int64_t slot_bytes;
  char *host_bricks;       // pinned, nbricks * slot_bytes
  float2 *minmax_dev;      // nbricks
  int32_t F;               // skip-block edge (min(E, 16)): blocks of F^3 inside each brick
  int32_t fnbx, fnby, fnbz;
  int64_t nfine;
  float2 *fine_minmax_dev; // nfine
  uint32_t *fine_bits_dev; // occupancy bits + radius plane, rebuilt per render
  bool fine_radius;        // the radius plane can be built for the fine grid
  uint8_t *occ_dev;
  uint8_t *occ_host;       // pinned
  int32_t *page_dev[2];    // per pool half (streaming) or [0] (all resident)
  int32_t *page_host[2];   // pinned
  hipStream_t copy_stream; // brick copies while the render stream renders
  hipEvent_t copied[2], rendered[2];
  bool copied_rec[2], rendered_rec[2];
  char *pool;
  int64_t nslots;
  std::vector<int64_t> slot_brick;  // slot -> brick or -1
  std::vector<int64_t> brick_slot;  // brick -> slot or -1
  float4 *state;
  int32_t *next;
  int64_t state_cap;
  vr_bricked_stats stats;
};

namespace vr {

static inline int64_t clampl(int64_t a, int64_t lo, int64_t hi) { return a < lo ? lo : (a > hi ? hi : a); }

// Copy brick (bx, by, bz)'s footprint into dst (S^3 elements from bE - 1 on
// each axis, x fastest, edge-clamped) and return the (min, max) of the
// footprint proper, [bE-1, bE+E+1] (the extra last plane does not count).
template <class T>
static float2 gather_brick(const T *src, int64_t nx, int64_t ny, int64_t nz, int E, int S, int64_t bx, int64_t by,
                           int64_t bz, T *dst) {
  float mn = INFINITY, mx = -INFINITY;
  const int64_t ox = bx * E - 1, oy = by * E - 1, oz = bz * E - 1;
  for (int zl = 0; zl < S; ++zl) {
    const int64_t z = clampl(oz + zl, 0, nz - 1);
    for (int yl = 0; yl < S; ++yl) {
      const int64_t y = clampl(oy + yl, 0, ny - 1);
      const T *row = src + (z * ny + y) * nx;
      T *out = dst + ((int64_t)zl * S + yl) * S;
      for (int xl = 0; xl < S; ++xl) {
        const T v = row[clampl(ox + xl, 0, nx - 1)];
        out[xl] = v;
        if (xl <= E + 2 && yl <= E + 2 && zl <= E + 2) {
          const float f = (float)v;
          mn = f < mn ? f : mn;
          mx = f > mx ? f : mx;
        }
      }
    }
  }
  return make_float2(mn, mx);
}

// (min, max) of every skip block of edge F inside brick (bx, by, bz), over
// its footprint [fF-1, fF+F+1] per axis, read from the brick's gathered
// (edge-clamped) footprint; out[] is indexed like the fine grid.
template <class T>
static void fine_minmax(const T *slot, int E, int S, int F, int64_t bx, int64_t by, int64_t bz, int32_t fnbx,
                        int32_t fnby, int32_t fnbz, float2 *out) {
  const int per = E / F;
  for (int fk = 0; fk < per; ++fk)
    for (int fj = 0; fj < per; ++fj)
      for (int fi = 0; fi < per; ++fi) {
        const int64_t gx = bx * per + fi, gy = by * per + fj, gz = bz * per + fk;
        if (gx >= fnbx || gy >= fnby || gz >= fnbz) continue;
        float mn = INFINITY, mx = -INFINITY;
        // slot-local footprint: [fi F, fi F + F + 2] (the slot starts at bE - 1)
        for (int z = fk * F; z <= fk * F + F + 2; ++z)
          for (int y = fj * F; y <= fj * F + F + 2; ++y) {
            const T *row = slot + ((int64_t)z * S + y) * S;
            for (int x = fi * F; x <= fi * F + F + 2; ++x) {
              const float f = (float)row[x];
              mn = f < mn ? f : mn;
              mx = f > mx ? f : mx;
            }
          }
        out[gx + (int64_t)fnbx * (gy + (int64_t)fnby * gz)] = make_float2(mn, mx);
      }
}

// Front-to-back rank of brick (i, j, k) for a camera (see the file comment).
static int64_t brick_rank(const CamConst &c, int E, int64_t i, int64_t j, int64_t k) {
  const int64_t idx[3] = {i, j, k};
  int64_t r = 0;
  for (int a = 0; a < 3; ++a) {
    if (c.proj != 0) {
      const int64_t e = (int64_t)std::floor(c.eye[a] / (double)E);
      r += std::llabs(idx[a] - e);
    } else {
      const double d = c.fwd[a];
      r += d > 0.0 ? idx[a] : (d < 0.0 ? -idx[a] : 0);
    }
  }
  return r;
}

static void order_bricks(const CamConst &c, int E, int32_t nbx, int32_t nby, int32_t nbz, const uint8_t *occ,
                         std::vector<int64_t> &out) {
  std::vector<std::pair<int64_t, int64_t>> keyed;
  const int64_t nb = (int64_t)nbx * nby * nbz;
  keyed.reserve((size_t)nb);
  for (int64_t b = 0; b < nb; ++b) {
    if (occ && !occ[b]) continue;
    const int64_t i = b % nbx, j = (b / nbx) % nby, k = b / ((int64_t)nbx * nby);
    keyed.emplace_back(brick_rank(c, E, i, j, k), b);
  }
  std::sort(keyed.begin(), keyed.end());
  out.clear();
  for (auto &kv : keyed) out.push_back(kv.second);
}

// The walk's grid: the volume's skip blocks of edge F (no data; occupancy
// bits attached per render).
static VolConst fine_grid(const vr_bricked *v) {
  VolConst f;
  f.data = nullptr;
  f.dtype = v->dtype;
  f.nx = (int32_t)v->nx;
  f.ny = (int32_t)v->ny;
  f.nz = (int32_t)v->nz;
  f.bytes = 0;
  f.minmax = v->fine_minmax_dev;
  f.nbx = v->fnbx;
  f.nby = v->fnby;
  f.nbz = v->fnbz;
  f.edge = v->F;
  f.edge_shift = __builtin_ctz((unsigned)v->F);
  f.row_even = (v->nx % 2) == 0 ? 1 : 0;
  return f;
}

// A device buffer released on its stream when it goes out of scope (after the
// work queued with it).
struct StreamBuffer {
  int32_t *p;
  hipStream_t s;
  ~StreamBuffer() {
    if (p) (void)hipFreeAsync(p, s);
  }
};

static void destroy(vr_bricked *v) {
  if (!v) return;
  if (v->host_bricks) (void)hipHostFree(v->host_bricks);
  if (v->occ_host) (void)hipHostFree(v->occ_host);
  for (int h = 0; h < 2; ++h) {
    if (v->page_host[h]) (void)hipHostFree(v->page_host[h]);
    (void)hipFree(v->page_dev[h]);
    if (v->copied[h]) (void)hipEventDestroy(v->copied[h]);
    if (v->rendered[h]) (void)hipEventDestroy(v->rendered[h]);
  }
  if (v->copy_stream) (void)hipStreamDestroy(v->copy_stream);
  (void)hipFree(v->minmax_dev);
  (void)hipFree(v->fine_minmax_dev);
  (void)hipFree(v->fine_bits_dev);
  (void)hipFree(v->occ_dev);
  if (v->arena) {
    if (v->arena->owner == v) v->arena->owner = nullptr;
  } else {
    (void)hipFree(v->pool);
  }
  (void)hipFree(v->state);
  (void)hipFree(v->next);
  delete v;
}

}  // namespace vr

using namespace vr;

namespace vr {

// Device bytes a bricked volume holds besides its pool: block and skip-block
// ranges, occupancy, page tables, occupancy bits.
BrickArena *brick_arena_new(char *mem, uint64_t bytes) {
  BrickArena *a = new (std::nothrow) BrickArena();
  if (a) {
    a->mem = mem;
    a->bytes = bytes;
  }
  return a;
}

void brick_arena_delete(BrickArena *a) { delete a; }

uint64_t bricked_device_bytes(const vr_bricked *v) {
  const VolConst f = fine_grid(v);
  return (uint64_t)v->nbricks * (sizeof(float2) + 1 + 2 * sizeof(int32_t)) + (uint64_t)v->nfine * sizeof(float2) +
         occupancy_bytes(f);
}

vr_status bricked_create(const vr_volume *host_vol, int32_t brick_edge, uint64_t pool_bytes, BrickArena *arena,
                         vr_bricked **out) {
  if (!out) return fail(VR_E_INVALID_ARG, "out is NULL");
  *out = nullptr;
  if (!host_vol || !host_vol->data) return fail(VR_E_INVALID_ARG, "host volume or its data is NULL");
  if (host_vol->dtype != VR_U16 && host_vol->dtype != VR_I16 && host_vol->dtype != VR_F32)
    return fail(VR_E_INVALID_ARG, "unknown volume dtype %d", host_vol->dtype);
  if (host_vol->nx <= 0 || host_vol->ny <= 0 || host_vol->nz <= 0 || host_vol->nx > (1 << 20) ||
      host_vol->ny > (1 << 20) || host_vol->nz > (1 << 20))
    return fail(VR_E_INVALID_ARG, "volume dims must be in [1, 2^20]");
  if (brick_edge < 8 || brick_edge > 128 || (brick_edge & (brick_edge - 1)) != 0)
    return fail(VR_E_INVALID_ARG, "brick edge %d is not a power of two in [8, 128]", brick_edge);
  vr_bricked *v = new (std::nothrow) vr_bricked();
  if (!v) return fail(VR_E_OOM, "host allocation failed");
  v->arena = arena;
  if (arena) pool_bytes = arena->bytes;
  v->dtype = host_vol->dtype;
  v->nx = host_vol->nx;
  v->ny = host_vol->ny;
  v->nz = host_vol->nz;
  v->E = brick_edge;
  v->S = brick_edge + 4;  // the footprint E + 3 plus one plane: an even row length
  v->nbx = (int32_t)((v->nx + brick_edge - 1) / brick_edge);
  v->nby = (int32_t)((v->ny + brick_edge - 1) / brick_edge);
  v->nbz = (int32_t)((v->nz + brick_edge - 1) / brick_edge);
  v->nbricks = (int64_t)v->nbx * v->nby * v->nbz;
  v->F = std::min<int32_t>(brick_edge, 16);
  v->fnbx = (int32_t)((v->nx + v->F - 1) / v->F);
  v->fnby = (int32_t)((v->ny + v->F - 1) / v->F);
  v->fnbz = (int32_t)((v->nz + v->F - 1) / v->F);
  v->nfine = (int64_t)v->fnbx * v->fnby * v->fnbz;
  v->esz = v->dtype == VR_F32 ? 4 : 2;
  // 16 bytes of padding keep the kernel's 12-byte row windows inside the slot
  v->slot_bytes = (((int64_t)v->S * v->S * v->S * v->esz) + 16 + 255) & ~(int64_t)255;
  v->nslots = (int64_t)(pool_bytes / (uint64_t)v->slot_bytes);
  if (v->nslots < 1) {
    delete v;
    return fail(VR_E_INVALID_ARG, "pool of %llu bytes holds no brick of %lld bytes", (unsigned long long)pool_bytes,
                (long long)v->slot_bytes);
  }
  v->nslots = std::min<int64_t>(v->nslots, v->nbricks);
  hipError_t e = hipHostMalloc((void **)&v->host_bricks, (size_t)(v->nbricks * v->slot_bytes), hipHostMallocDefault);
  if (e != hipSuccess) {
    v->host_bricks = nullptr;
    destroy(v);
    return fail(VR_E_OOM, "pinned host allocation of %lld brick bytes: %s", (long long)(v->nbricks * v->slot_bytes),
                hipGetErrorString(e));
  }
  // gather every footprint (and its min/max, and its skip blocks' min/max)
  // with the host's threads
  std::vector<float2> mm((size_t)v->nbricks);
  std::vector<float2> fmm((size_t)v->nfine);
  const unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (unsigned t = 0; t < nt; ++t)
    pool.emplace_back([&, t]() {
      for (int64_t b = t; b < v->nbricks; b += nt) {
        const int64_t i = b % v->nbx, j = (b / v->nbx) % v->nby, k = b / ((int64_t)v->nbx * v->nby);
        char *dst = v->host_bricks + b * v->slot_bytes;
        if (v->dtype == VR_F32) {
          mm[b] = gather_brick((const float *)host_vol->data, v->nx, v->ny, v->nz, v->E, v->S, i, j, k, (float *)dst);
          fine_minmax((const float *)dst, v->E, v->S, v->F, i, j, k, v->fnbx, v->fnby, v->fnbz, fmm.data());
        } else if (v->dtype == VR_I16) {
          mm[b] = gather_brick((const int16_t *)host_vol->data, v->nx, v->ny, v->nz, v->E, v->S, i, j, k,
                               (int16_t *)dst);
          fine_minmax((const int16_t *)dst, v->E, v->S, v->F, i, j, k, v->fnbx, v->fnby, v->fnbz, fmm.data());
        } else {
          mm[b] = gather_brick((const uint16_t *)host_vol->data, v->nx, v->ny, v->nz, v->E, v->S, i, j, k,
                               (uint16_t *)dst);
          fine_minmax((const uint16_t *)dst, v->E, v->S, v->F, i, j, k, v->fnbx, v->fnby, v->fnbz, fmm.data());
        }
      }
    });
  for (auto &th : pool) th.join();
  const size_t nb = (size_t)v->nbricks;
  VolConst fvc = fine_grid(v);
  v->fine_radius = occupancy_planes_fit(fvc, VR_MAX_TF_NODES);
  if ((e = hipMalloc(&v->minmax_dev, nb * sizeof(float2))) != hipSuccess ||
      (e = hipMalloc(&v->fine_minmax_dev, (size_t)v->nfine * sizeof(float2))) != hipSuccess ||
      (e = hipMalloc(&v->fine_bits_dev, occupancy_bytes(fvc))) != hipSuccess ||
      (e = hipMalloc(&v->occ_dev, nb)) != hipSuccess ||
      (e = hipMalloc(&v->page_dev[0], nb * sizeof(int32_t))) != hipSuccess ||
      (e = hipMalloc(&v->page_dev[1], nb * sizeof(int32_t))) != hipSuccess ||
      (!arena && (e = hipMalloc(&v->pool, (size_t)(v->nslots * v->slot_bytes))) != hipSuccess)) {
    destroy(v);
    return fail(VR_E_OOM, "device allocation for the brick pool: %s", hipGetErrorString(e));
  }
  if ((e = hipHostMalloc((void **)&v->occ_host, nb, hipHostMallocDefault)) != hipSuccess ||
      (e = hipHostMalloc((void **)&v->page_host[0], nb * sizeof(int32_t), hipHostMallocDefault)) != hipSuccess ||
      (e = hipHostMalloc((void **)&v->page_host[1], nb * sizeof(int32_t), hipHostMallocDefault)) != hipSuccess) {
    destroy(v);
    return fail(VR_E_OOM, "pinned host allocation: %s", hipGetErrorString(e));
  }
  if ((e = hipStreamCreateWithFlags(&v->copy_stream, hipStreamNonBlocking)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&v->copied[0], hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&v->copied[1], hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&v->rendered[0], hipEventDisableTiming)) != hipSuccess ||
      (e = hipEventCreateWithFlags(&v->rendered[1], hipEventDisableTiming)) != hipSuccess) {
    destroy(v);
    return hip_fail(e, "copy stream and events");
  }
  if ((e = hipMemcpy(v->minmax_dev, mm.data(), nb * sizeof(float2), hipMemcpyHostToDevice)) != hipSuccess ||
      (e = hipMemcpy(v->fine_minmax_dev, fmm.data(), (size_t)v->nfine * sizeof(float2), hipMemcpyHostToDevice)) !=
          hipSuccess) {
    destroy(v);
    return hip_fail(e, "copy brick min/max");
  }
  if (arena) v->pool = arena->mem;
  v->slot_brick.assign((size_t)v->nslots, -1);
  v->brick_slot.assign(nb, -1);
  memset(&v->stats, 0, sizeof(v->stats));
  v->stats.bricks_total = (uint64_t)v->nbricks;
  v->stats.pool_slots = (uint64_t)v->nslots;
  v->stats.brick_bytes = (uint64_t)v->slot_bytes;
  *out = v;
  return VR_OK;
}

}  // namespace vr

extern "C" {

vr_status vr_bricked_create(const vr_volume *host_vol, int32_t brick_edge, uint64_t pool_bytes, vr_bricked **out) {
  return bricked_create(host_vol, brick_edge, pool_bytes, nullptr, out);
}

vr_status vr_brick_order(const int64_t dims[3], int32_t brick_edge, const vr_camera *cam, int64_t *order_out,
                         int64_t n) {
  if (!dims || !cam || !order_out) return fail(VR_E_INVALID_ARG, "dims, camera or output is NULL");
  if (brick_edge < 1) return fail(VR_E_INVALID_ARG, "brick edge must be positive");
  if (dims[0] <= 0 || dims[1] <= 0 || dims[2] <= 0) return fail(VR_E_INVALID_ARG, "dims must be positive");
  CamConst c;
  vr_status s = check_camera(cam, &c);
  if (s) return s;
  const int32_t nbx = (int32_t)((dims[0] + brick_edge - 1) / brick_edge);
  const int32_t nby = (int32_t)((dims[1] + brick_edge - 1) / brick_edge);
  const int32_t nbz = (int32_t)((dims[2] + brick_edge - 1) / brick_edge);
  const int64_t nb = (int64_t)nbx * nby * nbz;
  if (n < nb) return fail(VR_E_INVALID_ARG, "output holds %lld entries, need %lld", (long long)n, (long long)nb);
  std::vector<int64_t> order;
  order_bricks(c, brick_edge, nbx, nby, nbz, nullptr, order);
  std::copy(order.begin(), order.end(), order_out);
  return VR_OK;
}

vr_status vr_bricked_render(vr_bricked *v, const vr_camera *cams, int32_t n_cams, const vr_tf *tf,
                            const vr_params *p, float *out_rgba, void *stream) {
  if (!v) return fail(VR_E_INVALID_ARG, "bricked volume is NULL");
  if (!tf || !p || !out_rgba) return fail(VR_E_INVALID_ARG, "tf, params or out_rgba is NULL");
  BrickedArgs a;
  memset(&a, 0, sizeof(a));
  vr_status s = check_tf_fields(tf->table, tf->K, tf->v0, tf->v1, &a.tf);
  if (s) return s;
  if ((s = check_march(p->step, p->ert_threshold, 1, &a.mc))) return s;
  if (p->filter != VR_FILTER_BSPLINE) return fail(VR_E_UNSUPPORTED, "out-of-core rendering uses the cubic B-spline only");
  if (!cams || n_cams <= 0) return fail(VR_E_INVALID_ARG, "need at least one camera");
  for (int32_t i = 0; i < n_cams; ++i) {
    if ((s = check_camera(&cams[i], nullptr))) return s;
    if (cams[i].width != cams[0].width || cams[i].height != cams[0].height)
      return fail(VR_E_INVALID_ARG, "all cameras must share one image size");
  }
  hipStream_t st = (hipStream_t)stream;
  const int64_t npix = (int64_t)cams[0].width * cams[0].height;
  hipError_t e;
  if (v->arena && v->arena->owner != v) {
    // another volume's bricks fill the shared pool: its copies and passes
    // must be over before ours overwrite the slots (its passes ran on this
    // stream: the server renders one out-of-core request at a time on one
    // stream), and none of our bricks are resident
    const vr_bricked *prev = v->arena->owner;
    if (prev && ((e = hipStreamSynchronize(prev->copy_stream)) != hipSuccess ||
                 (e = hipStreamSynchronize(st)) != hipSuccess))
      return hip_fail(e, "brick pool hand-over");
    std::fill(v->slot_brick.begin(), v->slot_brick.end(), -1);
    std::fill(v->brick_slot.begin(), v->brick_slot.end(), -1);
    v->copied_rec[0] = v->copied_rec[1] = v->rendered_rec[0] = v->rendered_rec[1] = false;
    v->arena->owner = v;
  }
  if (npix > v->state_cap) {
    (void)hipFree(v->state);
    (void)hipFree(v->next);
    v->state = nullptr;
    v->next = nullptr;
    v->state_cap = 0;
    if ((e = hipMalloc(&v->state, (size_t)npix * sizeof(float4))) != hipSuccess ||
        (e = hipMalloc(&v->next, (size_t)npix * sizeof(int32_t))) != hipSuccess)
      return fail(VR_E_OOM, "ray state allocation: %s", hipGetErrorString(e));
    v->state_cap = npix;
  }
  VolConst &vc = a.vol;
  vc.data = nullptr;
  vc.dtype = v->dtype;
  vc.nx = (int32_t)v->nx;
  vc.ny = (int32_t)v->ny;
  vc.nz = (int32_t)v->nz;
  vc.minmax = v->minmax_dev;
  vc.nbx = v->nbx;
  vc.nby = v->nby;
  vc.nbz = v->nbz;
  vc.edge = v->E;
  vc.edge_shift = __builtin_ctz((unsigned)v->E);
  // 1. occupancy under this TF: of the bricks (their order and residency) and
  // of the skip blocks (the walk's leaps)
  if ((e = launch_block_occupancy(vc, a.tf, v->occ_dev, st)) != hipSuccess) return hip_fail(e, "occupancy launch");
  a.fine = fine_grid(v);
  e = v->fine_radius ? launch_occupancy_planes(a.fine, a.tf, v->fine_bits_dev, st)
                     : launch_occupancy_bits(a.fine, a.tf, v->fine_bits_dev, st);
  if (e != hipSuccess) return hip_fail(e, "occupancy bits launch");
  a.fine.occ = v->fine_bits_dev;
  a.fine.occ_radius = v->fine_radius ? kEmptyRadiusMax : 0;
  if ((e = hipMemcpyAsync(v->occ_host, v->occ_dev, (size_t)v->nbricks, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return hip_fail(e, "occupancy readback");
  a.pool = v->pool;
  a.page = v->page_dev[0];
  a.occ = v->occ_dev;
  a.state = v->state;
  a.next = v->next;
  a.slot_bytes = v->slot_bytes;
  a.slot_edge = v->S;
  a.W = cams[0].width;
  a.H = cams[0].height;
  std::vector<int64_t> order;
  std::vector<char> in_pass((size_t)v->nbricks, 0);
  for (int32_t view = 0; view < n_cams; ++view) {
    check_camera(&cams[view], &a.cam);
    // the in-core kernel's centre-out order of the super-tiles, shared by the
    // passes of this view (raster order if it cannot be allocated)
    RenderArgs ra{};
    ra.vol = vc;
    ra.W = a.W;
    ra.H = a.H;
    ra.n_views = 1;
    ra.cams[0] = a.cam;
    const StreamBuffer tile_order{make_tile_order(ra, st), st};
    a.order = tile_order.p;
    // 2. front-to-back order of the occupied bricks
    order_bricks(a.cam, v->E, v->nbx, v->nby, v->nbz, v->occ_host, order);
    // 3. passes
    const int64_t nocc = (int64_t)order.size();
    if (nocc > v->nslots && v->nslots >= 2) {
      // streaming: passes of half a pool each, alternating halves; the copies
      // of a pass (on the copy stream) overlap the previous pass's rendering
      const int64_t half = v->nslots / 2;
      int64_t pos = 0;
      a.first = 1;
      for (int pass = 0; pos < nocc; ++pass) {
        const int h = pass & 1;
        const int64_t end = std::min(nocc, pos + half);
        // the page table of this half is free once its last copy has run
        if (v->copied_rec[h] && (e = hipEventSynchronize(v->copied[h])) != hipSuccess)
          return hip_fail(e, "page table reuse");
        // the slots of this half are free once the pass that read them has run
        if (v->rendered_rec[h] && (e = hipStreamWaitEvent(v->copy_stream, v->rendered[h], 0)) != hipSuccess)
          return hip_fail(e, "copy stream wait");
        int32_t *page = v->page_host[h];
        for (int64_t b = 0; b < v->nbricks; ++b) page[b] = -1;
        for (int64_t q = pos; q < end; ++q) {
          const int64_t b = order[q], sl = h * half + (q - pos);
          const int64_t old = v->slot_brick[(size_t)sl];
          if (old >= 0) v->brick_slot[(size_t)old] = -1;
          const int64_t had = v->brick_slot[(size_t)b];
          if (had >= 0) v->slot_brick[(size_t)had] = -1;
          e = hipMemcpyAsync(v->pool + sl * v->slot_bytes, v->host_bricks + b * v->slot_bytes, (size_t)v->slot_bytes,
                             hipMemcpyHostToDevice, v->copy_stream);
          if (e != hipSuccess) return hip_fail(e, "brick upload");
          v->brick_slot[(size_t)b] = sl;
          v->slot_brick[(size_t)sl] = b;
          v->stats.bricks_uploaded++;
          v->stats.bytes_uploaded += (uint64_t)v->slot_bytes;
          page[b] = (int32_t)sl;
        }
        e = hipMemcpyAsync(v->page_dev[h], page, (size_t)v->nbricks * sizeof(int32_t), hipMemcpyHostToDevice,
                           v->copy_stream);
        if (e != hipSuccess || (e = hipEventRecord(v->copied[h], v->copy_stream)) != hipSuccess)
          return hip_fail(e, "page table upload");
        v->copied_rec[h] = true;
        if ((e = hipStreamWaitEvent(st, v->copied[h], 0)) != hipSuccess) return hip_fail(e, "render stream wait");
        a.page = v->page_dev[h];
        if ((e = launch_bricked_pass(a, st)) != hipSuccess) return hip_fail(e, "pass launch");
        if ((e = hipEventRecord(v->rendered[h], st)) != hipSuccess) return hip_fail(e, "pass event");
        v->rendered_rec[h] = true;
        v->stats.passes++;
        a.first = 0;
        pos = end;
      }
    } else {
      // every occupied brick fits (or the pool holds a single brick): passes
      // over the whole pool on the render stream, resident bricks reused
      int64_t pos = 0;
      a.first = 1;
      a.page = v->page_dev[0];
      do {
        const int64_t end = std::min(nocc, pos + v->nslots);
        for (int64_t q = pos; q < end; ++q) in_pass[(size_t)order[q]] = 1;
        // free the slots of resident bricks outside this pass
        std::vector<int64_t> free_slots;
        for (int64_t sl = 0; sl < v->nslots; ++sl) {
          const int64_t b = v->slot_brick[(size_t)sl];
          if (b >= 0 && !in_pass[(size_t)b]) {
            v->brick_slot[(size_t)b] = -1;
            v->slot_brick[(size_t)sl] = -1;
          }
          if (v->slot_brick[(size_t)sl] < 0) free_slots.push_back(sl);
        }
        // the previous page-table copy has been consumed once the stream is idle
        if ((e = hipStreamSynchronize(st)) != hipSuccess) return hip_fail(e, "pass synchronisation");
        int32_t *page = v->page_host[0];
        for (int64_t b = 0; b < v->nbricks; ++b) page[b] = -1;
        size_t fi = 0;
        for (int64_t q = pos; q < end; ++q) {
          const int64_t b = order[q];
          int64_t sl = v->brick_slot[(size_t)b];
          if (sl < 0) {
            sl = free_slots[fi++];
            e = hipMemcpyAsync(v->pool + sl * v->slot_bytes, v->host_bricks + b * v->slot_bytes,
                               (size_t)v->slot_bytes, hipMemcpyHostToDevice, st);
            if (e != hipSuccess) return hip_fail(e, "brick upload");
            v->brick_slot[(size_t)b] = sl;
            v->slot_brick[(size_t)sl] = b;
            v->stats.bricks_uploaded++;
            v->stats.bytes_uploaded += (uint64_t)v->slot_bytes;
          }
          page[b] = (int32_t)sl;
        }
        e = hipMemcpyAsync(v->page_dev[0], page, (size_t)v->nbricks * sizeof(int32_t), hipMemcpyHostToDevice, st);
        if (e != hipSuccess) return hip_fail(e, "page table upload");
        if ((e = launch_bricked_pass(a, st)) != hipSuccess) return hip_fail(e, "pass launch");
        v->stats.passes++;
        a.first = 0;
        for (int64_t q = pos; q < end; ++q) in_pass[(size_t)order[q]] = 0;
        pos = end;
      } while (pos < nocc);
    }
    v->stats.bricks_occupied = (uint64_t)nocc;
    // 4. image
    float4 *dst = reinterpret_cast<float4 *>(out_rgba) + (size_t)view * (size_t)npix;
    if ((e = launch_bricked_finish(v->state, dst, npix, st)) != hipSuccess) return hip_fail(e, "finish launch");
  }
  uint64_t resident = 0;
  for (int64_t sl = 0; sl < v->nslots; ++sl) resident += v->slot_brick[(size_t)sl] >= 0;
  v->stats.bricks_resident = resident;
  return VR_OK;
}

vr_status vr_bricked_stats_get(const vr_bricked *v, vr_bricked_stats *out) {
  if (!v || !out) return fail(VR_E_INVALID_ARG, "bricked volume or output is NULL");
  *out = v->stats;
  return VR_OK;
}

void vr_bricked_free(vr_bricked *v) {
  if (v) (void)hipDeviceSynchronize();
  destroy(v);
}

}  // extern "C"
