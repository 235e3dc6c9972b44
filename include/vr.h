/*
 * vr.h -- C ABI of the MI355X (gfx950) tricubic volume ray caster.
 *
 * The calls follow the paper's statement of the problem (Section 2,
 * "Methodology", the ray-casting paragraph before Fig. 2): a volume, a
 * camera (the observer's position and a ray direction per pixel), a step
 * with which the ray moves, and a transfer function T(V) that maps a value
 * to colour and opacity (Fig. 3 discussion) go in; an RGBA image comes out.
 * Reconstruction is the cubic spline the paper adopts (Section 2, Fig. 4
 * discussion), classification happens after interpolation
 * (post-classification), rays stop early once opaque and blocks holding
 * nothing visible are skipped ("Pros" (b) of the block-decomposition
 * analysis).
 *
 * Conventions shared by every call:
 *   - Index space.  Voxel (i, j, k) is centred at (i, j, k); the volume
 *     occupies the box [-1/2, n-1/2] on each axis.  Memory order is x
 *     fastest, then y, then z.  Addresses outside the grid read the nearest
 *     edge voxel.  Voxel spacing is folded into the camera by the caller, so
 *     distances, the step and the extinction are in voxel units.
 *   - Memory.  Pointers documented as DEVICE are HIP device pointers on the
 *     current device, caller-owned unless stated otherwise.  Pointers
 *     documented as HOST are read before the call returns.
 *   - Streams.  `stream` is a hipStream_t (NULL = the default stream).  Work
 *     is enqueued asynchronously; nothing synchronises unless stated.
 *     Arguments are validated on the host before anything is enqueued.
 *   - Errors.  Every call returns a vr_status; no exception crosses the ABI.
 *     vr_last_error() gives a message for the calling thread's last non-OK
 *     status.  A device fault surfaces as VR_E_DEVICE at a later call.
 */
#ifndef VR_H
#define VR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define VR_ABI_VERSION 2

typedef enum {
    VR_OK = 0,
    VR_E_INVALID_ARG = 1, /* an argument failed validation; nothing was enqueued */
    VR_E_UNSUPPORTED = 2, /* valid but not supported (dtype, size limit)          */
    VR_E_OOM = 3,         /* a library allocation failed                           */
    VR_E_DEVICE = 4,      /* a HIP runtime call failed                             */
    VR_E_BUDGET = 5,      /* serving: the request can never fit the HBM budget     */
    VR_E_NOT_FOUND = 6,   /* serving: unknown volume id or ticket                  */
    VR_E_BUSY = 7,        /* serving: the volume has requests in flight            */
    VR_E_TIMEOUT = 8,     /* serving: wait timed out; the ticket stays valid        */
    VR_E_SHUTDOWN = 9     /* serving: the server was destroyed before completion   */
} vr_status;

typedef enum { VR_U16 = 0, VR_I16 = 1, VR_F32 = 2 } vr_dtype;

/* A scalar volume.  data: DEVICE, nx*ny*nz elements of `dtype`, dense, x
 * fastest, 4-byte aligned.  The CT data the paper renders are 12-bit values
 * stored in 16 bits (Section 2, Fig. 4 discussion); u16/i16 keep that
 * footprint, f32 serves real-valued (differentiable) grids. */
typedef struct {
    const void *data;
    int32_t dtype; /* vr_dtype */
    int32_t reserved;
    int64_t nx, ny, nz;
} vr_volume;

/* A camera: where the observer stands and, for every pixel, the direction
 * its ray leaves in (the ray-casting paragraph of Section 2).  All vectors
 * in index space; right/up/forward orthonormal.
 * Pixel (i, j), i the column and j the row, has centre (i+1/2, j+1/2) and
 *   sx = 2 (i + 1/2) / width - 1,   sy = 1 - 2 (j + 1/2) / height.
 * Perspective (projection 1): origin = eye,
 *   direction = normalize(forward + sx tan(fov_y/2) (width/height) right
 *                                 + sy tan(fov_y/2) up).
 * Orthographic (projection 0): origin = eye + sx (ortho_w/2) right
 *   + sy (ortho_h/2) up, direction = normalize(forward).
 * Ray setup is evaluated in FP64. */
typedef struct {
    int32_t projection; /* 0 orthographic, 1 perspective */
    int32_t width, height;
    int32_t reserved;
    double eye[3], right[3], up[3], forward[3];
    double fov_y;            /* radians, perspective only, in (0, pi) */
    double ortho_w, ortho_h; /* image-plane extent in voxels, orthographic only */
} vr_camera;

/* A transfer function T(V) (Section 2, Fig. 3 discussion): K nodes of
 * (r, g, b, sigma) fp32, node j at value v0 + j (v1 - v0) / (K - 1), linear
 * between nodes, the end nodes beyond [v0, v1].  r, g, b are emission colours;
 * sigma >= 0 is the extinction per voxel length, so a sample's opacity is
 * 1 - exp(-sigma step) (0 fully transparent, 1 opaque).
 * table: DEVICE, K*4 floats.  2 <= K <= VR_MAX_TF_NODES, v1 > v0.
 * Every entry must be finite and every sigma >= 0.  The host cannot read a
 * device table without waiting for the device, so the kernels check it as
 * they stage it: a call that meets an invalid table writes NaN to all of its
 * results (pixels, gradients, occupancy counts every block occupied) and
 * records the fault on the device; vr_device_status reports it. */
#define VR_MAX_TF_NODES 1024
typedef struct {
    const float *table;
    int32_t K;
    float v0, v1;
} vr_tf;

/* Marching parameters.
 *   step           in [1/1024, 1024] voxels.  The ray moves from its origin
 *                  with this step: samples sit at distances
 *                  t_k = (k + 1/2) step from the origin, for every integer
 *                  k >= 0 with t_in < t_k < t_out, where [t_in, t_out] is
 *                  the ray's intersection with the box (t_in clamped to 0).
 *                  Positions are computed from k, never accumulated; rays of
 *                  neighbouring pixels share sample distances.
 *   ert_threshold  early ray termination: a ray stops after the sample whose
 *                  accumulated opacity reaches the threshold; values outside
 *                  (0, 1) disable it.
 *   use_skip       nonzero: skip samples in blocks that cannot be visible
 *                  under the TF (needs a vr_blocks of this volume).  The
 *                  image is bit-identical to rendering without skipping.
 *   counters       optional DEVICE uint64_t[4] that the render ADDS to:
 *                  [0] evaluated samples, [1] lattice samples, [2] rays with
 *                  at least one lattice sample, [3] evaluated samples whose
 *                  taps were read from global memory rather than from an
 *                  LDS-staged box.  NULL = not counted. */
typedef struct {
    float step;
    float ert_threshold;
    int32_t use_skip;
    int32_t filter;      /* VR_FILTER_*; vr_render only, 0 elsewhere */
    uint64_t *counters;
} vr_params;

/* Reconstruction filters (the paper's filter comparison, Fig. 4 discussion).
 * VR_FILTER_BSPLINE: the uniform cubic B-spline (the default reading).
 * VR_FILTER_CATMULL_ROM: the interpolating Catmull-Rom cubic on the same 64
 *   taps, weights (-t^3+2t^2-t)/2, (3t^3-5t^2+2)/2, (-3t^3+4t^2+t)/2,
 *   (t^3-t^2)/2.  Its samples can leave their taps' range by at most
 *   w = ((1 + 2/8)^3 - 1)/2 = 0.4765625 of it, so its block test widens every
 *   block's range to [lo - w (hi - lo), hi + w (hi - lo)] (fp32 fused
 *   multiply-adds) and skipping stays exact.
 * VR_FILTER_BSPLINE_PRECLASSIFIED: pre-classification with the cubic
 *   B-spline: every tap is classified first and the weights interpolate the
 *   opacity-weighted channels (sigma r, sigma g, sigma b, sigma); the sample's
 *   colour is the weighted colour over its extinction (0 where that is 0).
 *   Its extinction is zero exactly where every tap's is, so the plain block
 *   test stays exact.
 * VR_FILTER_TRILINEAR: the paper's baseline filter, weights (0, 1-t, t, 0)
 *   on the same stencil (exact skipping with the plain block test).
 * (The interpolating cubic B-spline is vr_prefilter_bspline + the default.) */
#define VR_FILTER_BSPLINE 0
#define VR_FILTER_CATMULL_ROM 1
#define VR_FILTER_BSPLINE_PRECLASSIFIED 2
#define VR_FILTER_TRILINEAR 3

/* ---------------------------------------------------------------------- */
/* Blocks: the auxiliary structure for empty-space leaping (Section 2,     */
/* block decomposition into overlapping fixed-size blocks with smaller     */
/* remainder blocks, Fig. 3; "Pros" (a) and (b)).                           */
/* ---------------------------------------------------------------------- */

/* Opaque, library-owned.  Holds, for every block b (grid ceil(n/E) per
 * axis, x-block fastest), the min and max voxel value over the block's
 * footprint: [bE-1, bE+E+1] per axis clamped to the grid, i.e. every voxel a
 * cubic-spline sample whose cell floor(p) lies in b can read (the paper's
 * overlap for cubic sampling).  It refers to the volume's memory, which must
 * stay alive and unchanged while the blocks are used. */
typedef struct vr_blocks vr_blocks;

/* Build the block min/max for `vol` with edge `block_edge` (a power of two
 * in [4, 64]).
 * Enqueued on `stream`; *out is valid immediately and usable on the same
 * stream.  Allocates device memory (16 bytes per block: the ranges and
 * their Catmull-Rom widening).
 * Errors: VR_E_INVALID_ARG (null/invalid volume, edge out of range),
 * VR_E_OOM, VR_E_DEVICE. */
vr_status vr_build_blocks(const vr_volume *vol, int32_t block_edge, void *stream, vr_blocks **out);

/* Block-grid dimensions (nbx, nby, nbz) and edge.  Host only. */
vr_status vr_blocks_info(const vr_blocks *blocks, int64_t dims_out[3], int32_t *edge_out);

/* Copy the per-block (min, max) as fp32 pairs, x-block fastest, into
 * dst_device (DEVICE, at least 2 * nblocks floats).  Values of 16-bit
 * volumes are exact.  Enqueued on `stream`. */
vr_status vr_blocks_minmax(const vr_blocks *blocks, float *dst_device, int64_t dst_count, void *stream);

/* TF-dependent occupancy of every block: occ_device[b] = 1 unless every TF
 * node in [floor(u(min_b)) - 1, ceil(u(max_b)) + 1] (clamped to [0, K-1])
 * has zero extinction, u(v) = (v - v0) * ((K-1) / (v1 - v0)) in fp32.  The
 * renderer takes the same decision on the fly.  occ_device: DEVICE, at least
 * nblocks bytes.  Enqueued on `stream`. */
vr_status vr_block_occupancy(const vr_blocks *blocks, const vr_tf *tf, uint8_t *occ_device, int64_t n,
                             void *stream);

void vr_blocks_free(vr_blocks *blocks);

/* ---------------------------------------------------------------------- */
/* Rendering.                                                              */
/* ---------------------------------------------------------------------- */

/* Render n_cams views (all the same width x height) of `vol`.
 * cams: HOST array of n_cams cameras.  tf, p: HOST structs.
 * blocks: required when p->use_skip, built from this volume; else may be NULL.
 * out_rgba: DEVICE, n_cams * height * width * 4 floats, [view][row][col][rgba],
 *   written in full: premultiplied (C_r, C_g, C_b, 1 - T) over transparent
 *   black; rays that miss the box give (0, 0, 0, 0).
 * Per ray: front-to-back C += T a c, T *= 1 - a with a = 1 - exp(-sigma step),
 * starting from C = 0, T = 1.
 * Errors: VR_E_INVALID_ARG (null pointers, non-finite camera, sizes <= 0,
 * step out of range, K out of range, v1 <= v0, skip without blocks or with blocks of
 * another volume), VR_E_DEVICE. */
vr_status vr_render(const vr_volume *vol, const vr_blocks *blocks, const vr_camera *cams, int32_t n_cams,
                    const vr_tf *tf, const vr_params *p, float *out_rgba, void *stream);

/* vr_render for callers that cannot allocate device memory: code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation.
 * Arguments, results and errors as vr_render (the image is bit-identical);
 * nothing is allocated: the per-launch workgroup order and the occupancy
 * planes of the block grid live in a 2 MiB (+ 1 KiB) scratch array the library keeps
 * in device memory on every GPU it runs on (until the process ends).
 * Limits: a view of at most 262,144 16x16 tiles (8192 x 8192 pixels; views
 * are launched as many at a time as the scratch orders), and with
 * use_skip at most 2,796,192 blocks (1 MiB of occupancy planes); beyond them
 * VR_E_INVALID_ARG, nothing enqueued.  Every call on one GPU uses that GPU's
 * array: calls that overlap on one GPU (other streams, other threads) race,
 * so serialise them.  Every scratch entry a launch reads is written by that
 * launch first. */
vr_status vr_render_noalloc(const vr_volume *vol, const vr_blocks *blocks, const vr_camera *cams, int32_t n_cams,
                            const vr_tf *tf, const vr_params *p, float *out_rgba, void *stream);

/* Interpolating cubic B-spline.  The paper compares reconstruction filters
 * (Section 2, the filter comparison of Fig. 4); the plain cubic B-spline
 * smooths, its prefiltered form interpolates.  Writes to coeff_out (DEVICE,
 * nx*ny*nz fp32, layout of the volume; may not alias vol->data) the
 * coefficients c whose B-spline reconstruction (clamp-to-edge addressing)
 * passes through every voxel value: along every axis line
 *   (c[i-1] + 4 c[i] + c[i+1]) / 6 = v[i],  c[-1] = c[0], c[n] = c[n-1],
 * solved along x, then y, then z (fp32 elimination with FP64-derived
 * pivots).  Render the coefficient volume (VR_F32) with vr_render; its
 * vr_build_blocks min/max bound the reconstructed values exactly, so skipping
 * stays exact.  Enqueued on `stream` (the host waits once for a small pivot
 * table).  Errors: VR_E_INVALID_ARG, VR_E_UNSUPPORTED, VR_E_OOM, VR_E_DEVICE. */
vr_status vr_prefilter_bspline(const vr_volume *vol, float *coeff_out, void *stream);

/* Local lighting.  The paper lights its renderings with Phong's model, the
 * gradient for the normal taken with the same cubic filter as the value
 * (Section 2, the paragraph on the three-voxel block overlap).  Here every
 * sample's classified colour c becomes
 *   c' = c (ambient + diffuse |n.L|) + specular |n.H|^shininess
 * (Phong's model in the Blinn half-vector form, lit from both sides), where
 *   g = the analytic gradient of the tricubic B-spline reconstruction at the
 *       sample (derivative weights on the same 64 taps), in value units per
 *       voxel;
 *   n = -g / max(|g|, grad_min): the unit normal where |g| >= grad_min,
 *       shrinking to zero below (flat regions take ambient light only);
 *   V = -(ray direction); L = V for a headlight, else `light` normalised;
 *   H = (L + V) / |L + V|, and no specular term when L = -V.
 * Opacity, early termination and skipping are those of the unlit render. */
typedef struct {
    float ambient, diffuse, specular; /* finite, >= 0                           */
    float shininess;                  /* in [1, 1024]                           */
    float light[3];                   /* towards the light, any nonzero length  */
    int32_t headlight;                /* nonzero: light at the eye; light unused */
    float grad_min;                   /* finite, > 0                            */
    int32_t reserved;
} vr_shading;

/* vr_render with local lighting (`shading`: HOST struct, read before the call
 * returns).  Arguments, layout and errors as vr_render, plus
 * VR_E_INVALID_ARG for a NULL or out-of-range shading.  There is no adjoint
 * of the lit render (vr_render_backward differentiates the unlit model). */
vr_status vr_render_shaded(const vr_volume *vol, const vr_blocks *blocks, const vr_camera *cams, int32_t n_cams,
                           const vr_tf *tf, const vr_params *p, const vr_shading *shading, float *out_rgba,
                           void *stream);

/* Pre-integrated classification.  The paper combines its ray caster with
 * tables of previously integrated rendering (Section 2, the proposed method;
 * the conclusion's pre-integrated rendering against sampling artefacts).
 * A segment of length `step` along which the value rises linearly from TF
 * node i to node j has, with u(x) = i + (j - i) x / step and
 * tau(x) = integral_0^x sigma(u) dx',
 *   alpha(i, j) = 1 - exp(-tau(step)),
 *   C(i, j)     = integral_0^step c(u(x)) sigma(u(x)) exp(-tau(x)) dx
 * (premultiplied).  The table holds (C_r, C_g, C_b, alpha) for every node
 * pair, integrated in FP64 (pieces between node crossings, Gauss-Legendre on
 * sub-intervals of optical depth <= 1/32) and stored as fp32.
 * Opaque, library-owned; it remembers the TF (pointer, K, v0, v1) and step it
 * was built for.  A table built from an invalid TF is all NaN (see vr_tf). */
typedef struct vr_preint vr_preint;

/* Build the K x K table for `tf` (HOST struct; its DEVICE table is read by
 * the enqueued kernel) and `step` (range of vr_params.step).  Enqueued on
 * `stream`; allocates K*K*16 bytes of device memory.
 * Errors: VR_E_INVALID_ARG, VR_E_OOM, VR_E_DEVICE. */
vr_status vr_preint_build(const vr_tf *tf, float step, void *stream, vr_preint **out);

/* Copy the table (K*K*4 floats, entry (i, j) at 4 (i K + j)) into dst_device
 * (DEVICE, at least K*K*4 floats).  Enqueued on `stream`. */
vr_status vr_preint_table(const vr_preint *table, float *dst_device, int64_t dst_count, void *stream);

void vr_preint_free(vr_preint *table);

/* Pre-integrated render.  The ray's lattice cells (cell k between t = k step
 * and (k+1) step, for the k whose midpoints are vr_render's samples) are the
 * segments: the value is reconstructed at every cell boundary (a boundary may
 * lie up to half a step outside the box; clamp-to-edge defines the field
 * there) and each cell takes the table's bilinear lookup at (u(front),
 * u(back)), u clamped to [0, K-1]; front to back C += T C_cell, T *= 1 -
 * alpha_cell; early termination after the cell whose opacity reaches the
 * threshold.  With use_skip, a cell is skipped iff no value in the union of
 * its two boundary points' block ranges can meet non-zero extinction (the
 * image is bit-identical to rendering every cell).
 * table: built by vr_preint_build from this tf (same table pointer, K, v0,
 * v1) and p->step, else VR_E_INVALID_ARG.  The TF contents must not have
 * changed since.  counters as vr_render with cells for samples ([3] counts
 * boundary values read from global memory).  Otherwise as vr_render. */
vr_status vr_render_preint(const vr_volume *vol, const vr_blocks *blocks, const vr_camera *cams, int32_t n_cams,
                           const vr_tf *tf, const vr_params *p, const vr_preint *table, float *out_rgba,
                           void *stream);

/* ---------------------------------------------------------------------- */
/* Out-of-core rendering: the paper's block decomposition of volumes that  */
/* do not fit GPU memory (Section 2: blocks overlapping by the voxels a    */
/* cubic stencil reads, smaller blocks at the far faces, empty blocks      */
/* excluded, blocks rendered in order from the observer; Fig. 3).          */
/* ---------------------------------------------------------------------- */

/* Opaque, library-owned: a volume kept in pinned host memory as bricks (the
 * footprint [bE-1, bE+E+1] per axis of every E^3 block, edge-clamped, stored
 * with one more plane per axis as (E+4)^3 voxels) plus a device pool of whole
 * bricks with a page table. */
typedef struct vr_bricked vr_bricked;

typedef struct {
    uint64_t passes;            /* rendering passes so far                     */
    uint64_t bricks_total;      /* bricks of the volume                        */
    uint64_t bricks_occupied;   /* occupied under the last TF                  */
    uint64_t bricks_uploaded;   /* host -> device brick copies so far          */
    uint64_t bytes_uploaded;
    uint64_t bricks_resident;   /* bricks in the pool after the last render    */
    uint64_t pool_slots;        /* bricks the pool holds                       */
    uint64_t brick_bytes;       /* bytes of one pool slot (brick + 16, to 256) */
} vr_bricked_stats;

/* Copy `host_vol` (its data is a HOST pointer here, read during the call
 * only; dims up to 2^20 per axis, no 4 GiB limit) into pinned host bricks of
 * edge `brick_edge` (a power of two in [8, 128]) with their min/max, and
 * allocate a device pool of floor(pool_bytes / brick bytes) bricks (at least
 * one).  Synchronous.  Errors: VR_E_INVALID_ARG, VR_E_OOM, VR_E_DEVICE. */
vr_status vr_bricked_create(const vr_volume *host_vol, int32_t brick_edge, uint64_t pool_bytes, vr_bricked **out);

/* Render n_cams views (one image size) of a bricked volume into out_rgba
 * (DEVICE, layout of vr_render).  Per view: the TF occupancy of every brick
 * (the test of vr_block_occupancy), the occupied bricks in front-to-back
 * order for the camera, then passes over consecutive runs of that order, as
 * many bricks as the pool holds (bricks already resident are reused, the
 * others copied from pinned memory on `stream`); each pass continues every
 * ray, in lattice order, through its bricks.  The image is bit-identical to
 * vr_render with skipping and blocks of the same edge (p->use_skip is
 * implied: empty bricks are never loaded).  The host waits for the stream
 * between passes (and once for the occupancy).  Not thread-safe per
 * vr_bricked.  Errors as vr_render, VR_E_OOM. */
vr_status vr_bricked_render(vr_bricked *bricked, const vr_camera *cams, int32_t n_cams, const vr_tf *tf,
                            const vr_params *p, float *out_rgba, void *stream);

vr_status vr_bricked_stats_get(const vr_bricked *bricked, vr_bricked_stats *out);

/* Front-to-back order of all bricks of edge `brick_edge` of a dims[0] x
 * dims[1] x dims[2] volume for `cam`: brick indices (x fastest) into
 * order_out (HOST, at least the brick count).  Host only; no device use.
 * Every ray of the camera meets its bricks in this order. */
vr_status vr_brick_order(const int64_t dims[3], int32_t brick_edge, const vr_camera *cam, int64_t *order_out,
                         int64_t n);

/* Waits for the device, then frees the pinned bricks and the pool. */
void vr_bricked_free(vr_bricked *bricked);

/* Adjoint of vr_render: gradients of L with respect to the voxel values and
 * the TF table, given g = dL/dRGBA.  Per ray the forward march is recomputed
 * front to back (no per-sample state is stored); the stopping sample of
 * early termination is held fixed.
 * out_rgba: DEVICE, the forward result of vr_render with the same arguments.
 * grad_rgba: DEVICE, same layout as out_rgba.
 * grad_volume: DEVICE fp32 nx*ny*nz or NULL; grad_tf: DEVICE fp32 K*4 or NULL.
 *   Both are OVERWRITTEN (zeroed, then accumulated with atomics, so the
 *   summation order is not deterministic).
 * Skipping is used only when grad_tf is NULL (zero-extinction nodes still
 * receive TF gradients).  When every sample is visited and `blocks` is given
 * (also with p->use_skip = 0; it must then have been built for `vol`), a
 * sample in a block that is empty under the TF and constant over its
 * footprint takes that constant as its value, without reconstruction, and
 * runs of such samples (which change neither colour nor transmittance) are
 * accounted for at once; the gradients equal those without `blocks` up to
 * summation order.  Errors as vr_render. */
vr_status vr_render_backward(const vr_volume *vol, const vr_blocks *blocks, const vr_camera *cams, int32_t n_cams,
                             const vr_tf *tf, const vr_params *p, const float *out_rgba, const float *grad_rgba,
                             float *grad_volume, float *grad_tf, void *stream);

/* ---------------------------------------------------------------------- */
/* Serving: volumes resident in HBM, many clients, continuous batching     */
/* (the paper's multi-client cloud service, Section 2 "Cloud architecture" */
/* and Section 3).                                                          */
/* ---------------------------------------------------------------------- */

typedef struct vr_server vr_server;

typedef struct {
    uint64_t hbm_budget_bytes; /* device bytes charged to the server: resident volumes
                                  (their caller-owned memory), block structures, result
                                  images and per-request occupancy buffers */
    int32_t max_inflight;      /* admitted requests at once (slots), >= 1             */
    int32_t max_batch_tiles;   /* 16x16-pixel work items per launch (0 = 2048)        */
    int32_t device;            /* HIP device ordinal                                  */
    int32_t reserved;
    uint64_t brick_pool_bytes; /* device pool shared by out-of-core volumes, taken
                                  from the budget at the first such volume (0: none) */
} vr_serve_config;

/* One request.  tf_table_host: HOST K*4 floats, copied at submit. */
typedef struct {
    int32_t volume_id;
    int32_t K;
    const float *tf_table_host;
    float tf_v0, tf_v1;
    vr_camera cam;
    float step, ert_threshold;
    int32_t use_skip;
    int32_t reserved;
} vr_request;

typedef struct {
    uint64_t submitted, admitted, completed, rejected, queued, inflight;
    uint64_t hbm_used, hbm_peak;
    uint64_t launches, tiles;
    double p50_ms, p99_ms, mean_ms, max_ms; /* arrival (submit) -> completion */
    double rays_per_s;                      /* completed pixels / busy wall time */
    double busy_s;                          /* wall time with work in flight     */
    uint64_t samples;                       /* evaluated samples of completed launches */
    double samples_per_s;                   /* samples / busy wall time          */
    uint64_t queued_max;                    /* longest queue since the reset     */
    double queued_mean;                     /* time-averaged queue length        */
    uint64_t resident_bytes;                /* volumes + blocks charged          */
} vr_serve_stats;

/* Create a server with its own scheduler thread and HIP streams. */
vr_status vr_serve_create(const vr_serve_config *cfg, vr_server **out);

/* Register a resident volume (caller keeps its memory alive until removal)
 * and build its blocks with edge `block_edge`.  The volume's bytes and its
 * blocks count against the budget (pooled result images are freed to make
 * room); VR_E_BUDGET when they do not fit.  *volume_id receives the id. */
vr_status vr_serve_add_volume(vr_server *s, const vr_volume *vol, int32_t block_edge, int32_t *volume_id);

/* Register an out-of-core volume: `host_vol` is a HOST volume (read during
 * the call only; no 4 GiB limit), kept as pinned host bricks of edge
 * `brick_edge` (a power of two in [8, 128]) as vr_bricked_create does, for
 * volumes larger than the HBM budget (the paper's block decomposition of
 * data beyond GPU memory, Section 2).  Its bricks take turns in the server's
 * brick pool (vr_serve_config.brick_pool_bytes, allocated at the first such
 * volume and charged to the budget); its block structures are charged too.
 * Requests on it are submitted like any other; they are admitted in the
 * same FIFO order, and a worker thread renders them one at a time, pass by
 * pass through the pool, while in-core requests keep batching.  The image is
 * bit-identical to vr_render of the volume with 16^3 skip blocks.
 * Errors: VR_E_INVALID_ARG (no brick pool configured, invalid volume or
 * edge), VR_E_BUDGET, VR_E_OOM, VR_E_DEVICE. */
vr_status vr_serve_add_host_volume(vr_server *s, const vr_volume *host_vol, int32_t brick_edge, int32_t *volume_id);

/* Unregister; VR_E_BUSY while requests on it are queued or in flight. */
vr_status vr_serve_remove_volume(vr_server *s, int32_t volume_id);

/* Non-blocking submit; *ticket identifies the request.  VR_E_BUDGET if the
 * request's device memory (result image + occupancy buffer) can never fit
 * next to the resident volumes and blocks, VR_E_NOT_FOUND for an unknown
 * volume, VR_E_INVALID_ARG for invalid fields (a non-finite TF entry or a
 * negative extinction included), VR_E_SHUTDOWN after destroy.  Admission is
 * FIFO; a queued request that can no longer fit (volumes were added since)
 * completes with VR_E_BUDGET instead of blocking the queue. */
vr_status vr_serve_submit(vr_server *s, const vr_request *req, uint64_t *ticket);

/* Wait up to timeout_us (negative = forever) for `ticket`.  On VR_OK,
 * *rgba_device points to the DEVICE result (height*width*4 floats, layout of
 * vr_render), valid until vr_serve_release.  The result is complete and
 * visible to every stream. */
vr_status vr_serve_wait(vr_server *s, uint64_t ticket, int64_t timeout_us, const float **rgba_device);

/* Return a completed ticket's image to the pool. */
vr_status vr_serve_release(vr_server *s, uint64_t ticket);

vr_status vr_serve_stats_get(vr_server *s, vr_serve_stats *out);

/* Reset latency/throughput statistics (counters of resident state stay). */
vr_status vr_serve_stats_reset(vr_server *s);

/* Stop the scheduler, cancel queued requests (their waits return
 * VR_E_SHUTDOWN), drain in-flight launches and free every server
 * allocation.  Volumes stay caller-owned. */
vr_status vr_serve_destroy(vr_server *s);

/* ---------------------------------------------------------------------- */

/* Waits for `stream`, then reports whether a kernel on the current device
 * has met an invalid transfer-function table since the last call
 * (VR_E_INVALID_ARG, and the record is cleared) or not (VR_OK).
 * Errors: VR_E_DEVICE. */
vr_status vr_device_status(void *stream);

/* A render allocates per call (stream-ordered) its blocks' occupancy bits
 * under the TF and its workgroup order; when one of them cannot be allocated
 * or built, the call still succeeds with the same image on a slower path
 * (occupancy decided from min/max on every block change; workgroups in
 * Morton order).  These counters, process-wide since load, say how often
 * that happened (vr_render_noalloc allocates nothing).  occupancy, order:
 * HOST, one uint64_t each.  Errors: VR_E_INVALID_ARG (null pointers). */
vr_status vr_fallback_counts(uint64_t *occupancy, uint64_t *order);

/* Message for the calling thread's last non-OK status ("" if none). */
const char *vr_last_error(void);

int vr_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* VR_H */
