// vr_internal.h -- host-side launch interface between the C ABI layer and the
// HIP kernels.  Not installed; the public interface is include/vr.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "vr.h"
#include "vr_device.h"

namespace vr {

// Arguments of the whole-image render kernels (one launch covers up to
// kMaxCamsPerLaunch views that share volume, TF and marching parameters).
struct RenderArgs {
  VolConst vol;
  TfConst tf;
  MarchConst mc;
  float *out;                      // RGBA of the first view of this launch
  unsigned long long *counters;    // optional [evaluated, lattice, hit, -]
  const int32_t *order;            // workgroup -> super-tile order, or nullptr
  int32_t W, H, n_views, chunk_edge;
  int32_t use_box;                 // stage volume boxes in LDS (set at launch)
  int32_t shaded;                  // nonzero: local lighting with `shade`
  int32_t filter;                  // VR_FILTER_*
  int32_t occ_lds_words;           // > 0: stage vol.occ in LDS (set at launch)
  uint32_t *queue;                 // wavefront work-queue counters, or nullptr (set at launch)
  int32_t queue_items;             // wavefront items per queue (set at launch)
  ShadeConst shade;
  CamConst cams[kMaxCamsPerLaunch];
};

struct BackwardArgs {
  RenderArgs r;
  const float *out_rgba;   // forward result of the first view of this launch
  const float *grad_rgba;  // dL/dRGBA of the first view of this launch
  float *grad_vol;         // nullptr or nx*ny*nz
  float *grad_tf;          // nullptr or K*4
  int32_t use_box;         // stage the grid-gradient scatter in LDS boxes
  int32_t pad;
};



// Out-of-core pass over one view: bricks of edge E (the blocks' footprints,
// (E+4)^3 voxels each: the footprint plus one plane) resident in pool slots
// listed by the page table.
struct BrickedArgs {
  VolConst vol;            // dims, brick grid, edge, edge_shift (no data)
  VolConst fine;           // the same volume's skip blocks (edge <= 16) with occupancy bits: the walk's grid
  TfConst tf;
  MarchConst mc;
  CamConst cam;
  const char *pool;        // slot i at pool + i * slot_bytes
  const int32_t *page;     // per brick: slot in this pass, or -1
  const uint8_t *occ;      // per brick: TF occupancy
  float4 *state;           // per pixel: (C_r, C_g, C_b, T)
  int32_t *next;           // per pixel: next lattice index, -1 when finished
  int64_t slot_bytes;
  int32_t slot_edge;       // E + 4 (even)
  int32_t W, H;
  int32_t first;           // initialise the ray state
  int32_t use_box;         // stage LDS value boxes from the slots (set at launch)
  const int32_t *order;    // workgroup -> super-tile (centre-out, as in core), or nullptr: raster order
};

// Largest dynamic LDS a workgroup may allocate on the current device.
uint32_t max_lds_per_workgroup();

// Chunk edge of the workgroup -> tile mapping (VR_CHUNK_EDGE overrides: 1, 2,
// 4 or 8).
int32_t chunk_edge_setting();

hipError_t launch_render(const RenderArgs &a, hipStream_t s);
// Words of a.vol.occ a render launch stages in LDS after `lds` bytes of
// other state (0: read from global memory).
int32_t occupancy_lds_words(const RenderArgs &a, uint32_t lds);
// Number of workgroups of a render launch of `a` (one per super-tile with an
// order, else the padded Morton grid).
int64_t render_grid(const RenderArgs &a);
// Centre-out workgroup order for the views of `a`: super-tiles sorted by
// their distance to the projection of the volume's centre (the tiles whose
// rays cross the most volume go first, so the longest tiles do not start
// last), followed by the zeroed counters of the wavefront work queues
// (kOrderQueueInts).  Allocated on `s` (stream-ordered); the caller frees it
// with hipFreeAsync after its launches.  nullptr when it cannot be allocated
// (the Morton mapping is used then).  One order serves one launch: the
// launch consumes its counters.
int32_t *make_tile_order(const RenderArgs &a, hipStream_t s);
// The same order and counters written into `order` (tile_order_count(a) +
// kOrderQueueInts entries, every one written), allocating nothing.
hipError_t launch_tile_order(const RenderArgs &a, int32_t *order, hipStream_t s);
int64_t tile_order_count(const RenderArgs &a);
// Workgroups of kernel `fn` the current device holds at once with `lds` bytes
// of LDS each (0 when it cannot be found out).
int64_t resident_workgroups(const void *fn, uint32_t lds);
hipError_t launch_render_backward(const BackwardArgs &a, hipStream_t s);
hipError_t launch_block_minmax(const VolConst &v, float2 *out, hipStream_t s);
hipError_t launch_block_occupancy(const VolConst &v, const TfConst &tf, uint8_t *occ, hipStream_t s);
// The same decisions packed 32 blocks to a word (ceil(nb / 32) words).
hipError_t launch_occupancy_bits(const VolConst &v, const TfConst &tf, uint32_t *bits, hipStream_t s);
// The occupancy bits and, after them, the 2-bit radius plane (ceil(nb / 16)
// words) in one launch; hipErrorInvalidValue when its LDS window does not fit
// (see occupancy_planes_fit; then only launch_occupancy_bits applies).
hipError_t launch_occupancy_planes(const VolConst &v, const TfConst &tf, uint32_t *bits, hipStream_t s);
bool occupancy_planes_fit(const VolConst &v, int K);
// Bytes of the occupancy bits plus the radius plane of a block grid.
inline size_t occupancy_bytes(const VolConst &v) {
  const int64_t nb = (int64_t)v.nbx * v.nby * v.nbz;
  return (size_t)(((nb + 31) / 32 + (nb + 15) / 16) * 4);
}
hipError_t launch_fill_zero(float *p, int64_t n, hipStream_t s);
// Catmull-Rom samples leave their taps' range by at most this fraction of it.
constexpr float kCatmullRomWiden = 0.4765625f;  // ((1 + 2/8)^3 - 1) / 2
hipError_t launch_widen_minmax(const float2 *in, float2 *out, int64_t n, float w, hipStream_t s);
// coef: per axis (x, y, z) 2 n floats: 1 / pivot[i], then the eliminated
// super-diagonal sup[i] of the prefilter's tridiagonal system.
hipError_t launch_prefilter(const VolConst &v, float *out, const float *coef, hipStream_t s);
hipError_t launch_bricked_pass(const BrickedArgs &a, hipStream_t s);
hipError_t launch_bricked_finish(const float4 *state, float4 *out, int64_t n, hipStream_t s);
hipError_t launch_preint_table(const float *tf, int K, float step, float4 *out, uint32_t *status, hipStream_t s);
hipError_t launch_render_preint(const RenderArgs &a, const float4 *tab, hipStream_t s);

// Serving: one work item is a 16x16 super-tile of one request slot.
struct ServeSlot {
  VolConst vol;
  TfConst tf;
  MarchConst mc;
  CamConst cam;
  float *out;
};

struct ServeItem {
  int32_t slot;
  int16_t sx, sy;
};

// Device memory a render may use instead of allocating: room for the
// workgroup order of one launch and for the occupancy planes of the volume's
// block grid.  Every entry a launch reads is written by that launch first.
struct RenderScratch {
  int32_t *order;
  int64_t order_ints;
  uint32_t *occ;
  size_t occ_bytes;
};

// Validate the arguments of vr_render-like calls and fill the launch
// arguments (cameras excluded); api.cpp.
vr_status prepare_render(const vr_volume *vol, const vr_blocks *blocks, const vr_camera *cams, int32_t n_cams,
                         const vr_tf *tf, const vr_params *p, RenderArgs *a);
// Render the views of `a` (all launches); with `scratch` nothing is
// allocated (the caller has checked that its sizes suffice).
vr_status render_views(RenderArgs &a, const vr_camera *cams, int32_t n_cams, float *out_rgba, void *stream,
                       const float4 *preint, const RenderScratch *scratch);

// Out-of-core volumes whose bricks share one device pool (bricked.cpp): the
// pool is the arena's; a volume that renders after another finds none of its
// bricks resident.  Renders of volumes sharing an arena must not overlap.
struct BrickArena;
vr_status bricked_create(const vr_volume *host_vol, int32_t brick_edge, uint64_t pool_bytes, BrickArena *arena,
                         vr_bricked **out);
uint64_t bricked_device_bytes(const vr_bricked *v);
BrickArena *brick_arena_new(char *mem, uint64_t bytes);
void brick_arena_delete(BrickArena *a);

#ifdef VR_TIMELINE
// Records of the last launch of the forward / the adjoint (render_fwd.hip,
// render_bwd.hip): copy up to `max` records into host memory after a device
// synchronisation; return the launch's record count, or -1.
int64_t timeline_copy_fwd(unsigned long long *host, int64_t max);
int64_t timeline_copy_bwd(unsigned long long *host, int64_t max);
#endif

// Device address of the current device's TF status word (device_state.hip),
// nullptr when it cannot be obtained.
uint32_t *tf_status_word();

// Device operations of the serving loop (serve.cpp).  The server makes every
// device call through one of these tables: serve_hip_ops() is the HIP one;
// a CPU stand-in lets the scheduler's host threads be checked on their own
// (ThreadSanitizer, no device).  Each returns hipSuccess or an error;
// event_query returns hipErrorNotReady while the event's work runs.
struct ServeOps {
  hipError_t (*device_count)(int *n);
  hipError_t (*set_device)(int device);
  hipError_t (*stream_create)(hipStream_t *s);
  hipError_t (*stream_destroy)(hipStream_t s);
  hipError_t (*stream_sync)(hipStream_t s);
  hipError_t (*event_create)(hipEvent_t *e);
  hipError_t (*event_destroy)(hipEvent_t e);
  hipError_t (*event_record)(hipEvent_t e, hipStream_t s);
  hipError_t (*event_query)(hipEvent_t e);
  hipError_t (*stream_wait)(hipStream_t s, hipEvent_t e);
  hipError_t (*dev_alloc)(void **p, size_t bytes);
  hipError_t (*dev_free)(void *p);
  hipError_t (*host_alloc)(void **p, size_t bytes);
  hipError_t (*host_free)(void *p);
  hipError_t (*copy_async)(void *dst, const void *src, size_t bytes, hipMemcpyKind kind, hipStream_t s);
  hipError_t (*occupancy)(const VolConst &v, const TfConst &tf, uint32_t *bits, bool radius, hipStream_t s);
  hipError_t (*launch_batch)(const ServeSlot *slots_dev, const ServeItem *items_dev, int32_t n_items,
                             int32_t max_tf_k, unsigned long long *samples, hipStream_t s);
  // build the blocks of a resident volume (complete on return) and fill vc
  // with the volume and block constants; free_blocks releases them
  vr_status (*build_blocks)(const vr_volume *vol, int32_t edge, vr_blocks **out, VolConst *vc);
  void (*free_blocks)(vr_blocks *b);
};
const ServeOps *serve_hip_ops();
vr_status serve_create_with_ops(const vr_serve_config *cfg, const ServeOps *ops, vr_server **out);

// Validation helpers of the ABI layer (api.cpp); each fills the kernel-side
// constants and records vr_last_error on failure.
vr_status fail(vr_status s, const char *fmt, ...);
vr_status hip_fail(hipError_t e, const char *what);
vr_status check_volume(const vr_volume *v, VolConst *out);
vr_status check_tf_fields(const void *table, int32_t K, float v0, float v1, TfConst *out);
vr_status check_camera(const vr_camera *c, CamConst *out);
vr_status check_march(float step, float ert, int32_t use_skip, MarchConst *out);
vr_status check_shading(const vr_shading *sh, ShadeConst *out);
vr_status attach_blocks(const vr_blocks *b, const vr_volume *v, VolConst *vc);

// `samples`: device counter the launch adds its evaluated samples to.
hipError_t launch_serve_batch(const ServeSlot *slots_dev, const ServeItem *items_dev, int32_t n_items,
                              int32_t max_tf_k, unsigned long long *samples, hipStream_t s);

}  // namespace vr
