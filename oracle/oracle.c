/*
 * oracle.c -- plain, slow FP64 CPU reference for tricubic direct volume ray
 * casting with post-classification, front-to-back compositing, early ray
 * termination and block empty-space skipping.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load this library.  It shares no code, header,
 * table or helper with the GPU library, and the GPU library never calls it.
 *
 * What is computed follows the paper's Section 2 ("Methodology"):
 *   - one ray per image pixel, from the observer along a direction, moving
 *     with a fixed step and accumulating the pixel colour (ray casting,
 *     Fig. 2 and the paragraph before it);
 *   - voxels are a translucent emitting/absorbing medium ("Voxel graphics");
 *   - the scalar is reconstructed at every sample with cubic-spline
 *     (tricubic) interpolation (Section 2, "In this work the cubic
 *     interpolation is being used"; Fig. 4 discussion);
 *   - the interpolated value is then classified through the transfer function
 *     T(V) (post-classification, Fig. 3/Fig. 4 discussion);
 *   - rays terminate early once opaque and blocks holding nothing visible are
 *     skipped ("Pros" (b) of the block-decomposition analysis).
 * The paper gives no formulas for any of these steps.  The readings used here
 * (voxel-centred geometry, midpoint sample lattice, uniform cubic B-spline,
 * node-centred piecewise-linear transfer function, extinction optical model,
 * inclusive termination test, per-sample block skip) are the textbook
 * emission-absorption discretisation; each is stated at the function that
 * implements it.
 *
 * Everything is FP64 except the block-occupancy decision, which the paper
 * leaves to the implementation and which is taken in FP32 so that the GPU and
 * the oracle take the same integer decision.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { OR_U16 = 0, OR_I16 = 1, OR_F32 = 2, OR_F64 = 3 };

typedef struct {
    const void *data;
    int dtype;
    long nx, ny, nz;
} or_vol;

/* Voxel (x, y, z) with every index clamped to the grid (clamp-to-edge). */
static double or_voxel(const or_vol *v, long x, long y, long z)
{
    if (x < 0) x = 0;
    if (x > v->nx - 1) x = v->nx - 1;
    if (y < 0) y = 0;
    if (y > v->ny - 1) y = v->ny - 1;
    if (z < 0) z = 0;
    if (z > v->nz - 1) z = v->nz - 1;
    long idx = x + v->nx * (y + v->ny * z);
    switch (v->dtype) {
    case OR_U16: return (double)((const uint16_t *)v->data)[idx];
    case OR_I16: return (double)((const int16_t *)v->data)[idx];
    case OR_F32: return (double)((const float *)v->data)[idx];
    default: return ((const double *)v->data)[idx];
    }
}

static long or_clampl(long a, long lo, long hi) { return a < lo ? lo : (a > hi ? hi : a); }

int oracle_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads of the following calls (the CPU baseline times one core too). */
void oracle_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Block min/max (the auxiliary structure for empty-space leaping).          */
/*                                                                           */
/* The paper splits the volume into fixed-size blocks with smaller remainder */
/* blocks at the far faces, overlapping their neighbours by the voxels a     */
/* cubic stencil reads (Section 2, block decomposition and Fig. 3).  Here    */
/* that becomes, for each block b along an axis, the voxel range a tricubic  */
/* sample with floor(p) in [bE, bE+E-1] can touch: [bE-1, bE+E+1], clamped   */
/* to the grid.  Brute force over that footprint.                            */
/* out: nbz*nby*nbx*2 doubles, (min, max) per block, x-block fastest.        */
/* ------------------------------------------------------------------------ */
int oracle_blocks(const void *data, int dtype, long nx, long ny, long nz, int edge, double *out)
{
    if (!data || !out || edge <= 0 || nx <= 0 || ny <= 0 || nz <= 0) return 1;
    or_vol v = {data, dtype, nx, ny, nz};
    long nbx = (nx + edge - 1) / edge, nby = (ny + edge - 1) / edge, nbz = (nz + edge - 1) / edge;
    long nb = nbx * nby * nbz;
#pragma omp parallel for schedule(dynamic, 4)
    for (long b = 0; b < nb; ++b) {
        long bx = b % nbx, by = (b / nbx) % nby, bz = b / (nbx * nby);
        long x0 = or_clampl(bx * edge - 1, 0, nx - 1), x1 = or_clampl(bx * edge + edge + 1, 0, nx - 1);
        long y0 = or_clampl(by * edge - 1, 0, ny - 1), y1 = or_clampl(by * edge + edge + 1, 0, ny - 1);
        long z0 = or_clampl(bz * edge - 1, 0, nz - 1), z1 = or_clampl(bz * edge + edge + 1, 0, nz - 1);
        double mn = INFINITY, mx = -INFINITY;
        for (long z = z0; z <= z1; ++z)
            for (long y = y0; y <= y1; ++y)
                for (long x = x0; x <= x1; ++x) {
                    double a = or_voxel(&v, x, y, z);
                    if (a < mn) mn = a;
                    if (a > mx) mx = a;
                }
        out[2 * b] = mn;
        out[2 * b + 1] = mx;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Block occupancy under a transfer function.                                */
/*                                                                           */
/* A block may be skipped only if nothing inside it can be visible (Section  */
/* 2, "Pros" (b): empty-space skipping with auxiliary structures).  With a   */
/* piecewise-linear TF and non-negative extinction, every value v of a       */
/* sample in the block lies in [min, max]; such a sample reads only TF nodes */
/* between floor(u(min)) and ceil(u(max)).  One node of margin on each side  */
/* absorbs rounding of v.  The block is empty iff every node in              */
/* [floor(u(min)) - 1, ceil(u(max)) + 1] (clamped to [0, K-1]) has zero      */
/* extinction.  u is evaluated in FP32 as (v - v0) * ((K-1) / (v1 - v0)).    */
/* occ: one byte per block (1 occupied, 0 empty).                            */
/* ------------------------------------------------------------------------ */
/* Can a value in [lo, hi] (fp32) meet non-zero extinction?  The test above. */
static int or_range_occupied(const float *tf, int K, float v0, float scale, float lo, float hi)
{
    float ulo = (lo - v0) * scale;
    float uhi = (hi - v0) * scale;
    if (ulo < -2.0f) ulo = -2.0f;
    if (ulo > (float)K + 1.0f) ulo = (float)K + 1.0f;
    if (uhi < -2.0f) uhi = -2.0f;
    if (uhi > (float)K + 1.0f) uhi = (float)K + 1.0f;
    long jlo = (long)floorf(ulo) - 1, jhi = (long)ceilf(uhi) + 1;
    jlo = or_clampl(jlo, 0, K - 1);
    jhi = or_clampl(jhi, 0, K - 1);
    for (long j = jlo; j <= jhi; ++j)
        if (tf[4 * j + 3] != 0.0f) return 1;
    return 0;
}

/* widen >= 0: the range tested is [lo - widen (hi - lo), hi + widen (hi -  */
/* lo)] in fp32 fused multiply-adds, for filters whose samples can leave     */
/* the range of their taps (Catmull-Rom: the sum of the negative weights of  */
/* the 4x4x4 tensor product is at most ((1 + 2/8)^3 - 1)/2 = 0.4765625).     */
int oracle_occupancy(const double *minmax, long nblocks, const float *tf, int K, float v0, float v1, float widen,
                     uint8_t *occ)
{
    if (!minmax || !tf || !occ || K < 2 || !(v1 > v0) || !(widen >= 0.0f)) return 1;
    float scale = (float)(K - 1) / (v1 - v0);
    for (long b = 0; b < nblocks; ++b) {
        float lo = (float)minmax[2 * b], hi = (float)minmax[2 * b + 1];
        if (widen > 0.0f) {
            float d = hi - lo;
            float wlo = fmaf(-widen, d, lo), whi = fmaf(widen, d, hi);
            lo = wlo;
            hi = whi;
        }
        occ[b] = (uint8_t)or_range_occupied(tf, K, v0, scale, lo, hi);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Camera -> ray for pixel (i, j) (Section 2: a ray is an origin, e.g. the   */
/* observer, and a direction, one per image pixel).                          */
/* cam: 16 doubles = projection, eye[3], right[3], up[3], forward[3], fov_y, */
/* ortho_w, ortho_h.  Pixel centre (i+1/2, j+1/2); sx = 2(i+1/2)/W - 1,      */
/* sy = 1 - 2(j+1/2)/H.  Perspective: o = eye, d = normalize(forward +       */
/* sx tan(fov/2) (W/H) right + sy tan(fov/2) up).  Orthographic: o = eye +   */
/* sx (ortho_w/2) right + sy (ortho_h/2) up, d = normalize(forward).         */
/* ------------------------------------------------------------------------ */
static void or_ray(const double *cam, int W, int H, long i, long j, double o[3], double d[3])
{
    double sx = 2.0 * ((double)i + 0.5) / (double)W - 1.0;
    double sy = 1.0 - 2.0 * ((double)j + 0.5) / (double)H;
    const double *eye = cam + 1, *r = cam + 4, *u = cam + 7, *f = cam + 10;
    if (cam[0] != 0.0) {
        double th = tan(0.5 * cam[13]);
        double a = sx * th * ((double)W / (double)H);
        double b = sy * th;
        for (int k = 0; k < 3; ++k) {
            o[k] = eye[k];
            d[k] = f[k] + a * r[k] + b * u[k];
        }
    } else {
        double a = sx * (0.5 * cam[14]);
        double b = sy * (0.5 * cam[15]);
        for (int k = 0; k < 3; ++k) {
            o[k] = eye[k] + a * r[k] + b * u[k];
            d[k] = f[k];
        }
    }
    double n = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    for (int k = 0; k < 3; ++k) d[k] = d[k] / n;
}

/* Clip the ray against the volume box [-1/2, n-1/2] per axis (voxel-centred */
/* grid).  Returns 0 on a miss, else the entry and exit parameters.          */
static int or_clip(const double o[3], const double d[3], long nx, long ny, long nz, double *tin,
                   double *tout)
{
    double lo[3] = {-0.5, -0.5, -0.5};
    double hi[3] = {(double)nx - 0.5, (double)ny - 0.5, (double)nz - 0.5};
    double t0 = -INFINITY, t1 = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] == 0.0) {
            if (o[a] < lo[a] || o[a] > hi[a]) return 0;
            continue;
        }
        double ta = (lo[a] - o[a]) / d[a];
        double tb = (hi[a] - o[a]) / d[a];
        if (ta > tb) {
            double s = ta;
            ta = tb;
            tb = s;
        }
        if (ta > t0) t0 = ta;
        if (tb < t1) t1 = tb;
    }
    double te = t0 > 0.0 ? t0 : 0.0;
    if (!(t1 > te)) return 0;
    *tin = te;
    *tout = t1;
    return 1;
}

/* Uniform cubic B-spline weights for the taps floor(p)-1 .. floor(p)+2 at   */
/* fractional offset f (the reading of "cubic spline interpolation").        */
static void or_bspline(double f, double w[4])
{
    double g = 1.0 - f;
    w[0] = g * g * g / 6.0;
    w[1] = (3.0 * f * f * f - 6.0 * f * f + 4.0) / 6.0;
    w[2] = (-3.0 * f * f * f + 3.0 * f * f + 3.0 * f + 1.0) / 6.0;
    w[3] = f * f * f / 6.0;
}

/* Catmull-Rom weights (the interpolating cubic of the paper's filter        */
/* comparison, Fig. 4 discussion) for the same four taps.  Two of them are   */
/* negative: a sample can leave the range of its taps.                      */
static void or_catmull_rom(double f, double w[4])
{
    w[0] = (-f * f * f + 2.0 * f * f - f) / 2.0;
    w[1] = (3.0 * f * f * f - 5.0 * f * f + 2.0) / 2.0;
    w[2] = (-3.0 * f * f * f + 4.0 * f * f + f) / 2.0;
    w[3] = (f * f * f - f * f) / 2.0;
}

/* Trilinear weights on the same four taps (the paper's baseline filter): the */
/* two nearest taps only.                                                    */
static void or_trilinear(double f, double w[4])
{
    w[0] = 0.0;
    w[1] = 1.0 - f;
    w[2] = f;
    w[3] = 0.0;
}

/* One reconstructed sample: the 64 taps, their weights and the value.      */
typedef struct {
    long tap[64];
    double wt[64];
    double v;
} or_sample;

/* Tricubic reconstruction at p: the explicit 64-term sum over the 4x4x4     */
/* stencil, clamp-to-edge addressing.                                        */
/* filter: 0 cubic B-spline, 1 Catmull-Rom, 3 trilinear.                    */
static void or_reconstruct_f(const or_vol *vol, const double p[3], or_sample *s, int filter)
{
    long ix = (long)floor(p[0]), iy = (long)floor(p[1]), iz = (long)floor(p[2]);
    double wx[4], wy[4], wz[4];
    void (*weights)(double, double *) = filter == 1 ? or_catmull_rom : (filter == 3 ? or_trilinear : or_bspline);
    weights(p[0] - (double)ix, wx);
    weights(p[1] - (double)iy, wy);
    weights(p[2] - (double)iz, wz);
    double v = 0.0;
    int n = 0;
    for (int c = 0; c < 4; ++c)
        for (int b = 0; b < 4; ++b)
            for (int a = 0; a < 4; ++a) {
                long x = or_clampl(ix - 1 + a, 0, vol->nx - 1);
                long y = or_clampl(iy - 1 + b, 0, vol->ny - 1);
                long z = or_clampl(iz - 1 + c, 0, vol->nz - 1);
                double w = wx[a] * wy[b] * wz[c];
                s->tap[n] = x + vol->nx * (y + vol->ny * z);
                s->wt[n] = w;
                v += w * or_voxel(vol, x, y, z);
                ++n;
            }
    s->v = v;
}

static void or_reconstruct(const or_vol *vol, const double p[3], or_sample *s) { or_reconstruct_f(vol, p, s, 0); }

/* Derivative with respect to f of the four B-spline weights above: the     */
/* paper computes the gradient for local lighting with the same cubic       */
/* filter (Section 2, the three-voxel block overlap paragraph), i.e. the    */
/* gradient of the reconstructed field itself.                             */
static void or_bspline_deriv(double f, double d[4])
{
    double g = 1.0 - f;
    d[0] = -g * g / 2.0;
    d[1] = (9.0 * f * f - 12.0 * f) / 6.0;
    d[2] = (-9.0 * f * f + 6.0 * f + 3.0) / 6.0;
    d[3] = f * f / 2.0;
}

/* Analytic gradient of the tricubic reconstruction at p: per axis, the     */
/* explicit 64-term sum with that axis' weights replaced by derivative      */
/* weights (clamp-to-edge addressing as in the value).                      */
static void or_gradient(const or_vol *vol, const double p[3], double g[3])
{
    long ix = (long)floor(p[0]), iy = (long)floor(p[1]), iz = (long)floor(p[2]);
    double w[3][4], dw[3][4];
    long base[3] = {ix, iy, iz};
    for (int a = 0; a < 3; ++a) {
        or_bspline(p[a] - (double)base[a], w[a]);
        or_bspline_deriv(p[a] - (double)base[a], dw[a]);
    }
    g[0] = g[1] = g[2] = 0.0;
    for (int c = 0; c < 4; ++c)
        for (int b = 0; b < 4; ++b)
            for (int a = 0; a < 4; ++a) {
                long x = or_clampl(ix - 1 + a, 0, vol->nx - 1);
                long y = or_clampl(iy - 1 + b, 0, vol->ny - 1);
                long z = or_clampl(iz - 1 + c, 0, vol->nz - 1);
                double V = or_voxel(vol, x, y, z);
                g[0] += dw[0][a] * w[1][b] * w[2][c] * V;
                g[1] += w[0][a] * dw[1][b] * w[2][c] * V;
                g[2] += w[0][a] * w[1][b] * dw[2][c] * V;
            }
}

/* Local lighting (Section 2: Phong's model, with the gradient of the      */
/* cubic reconstruction as the surface normal).  shade = 9 doubles: ka, kd, */
/* ks, shininess, light direction (3, towards the light, any length),      */
/* headlight flag (nonzero: the light sits at the eye), grad_min.          */
/* The sample colour c becomes                                              */
/*   c (ka + kd |n.L|) + ks |n.H|^shininess                                 */
/* with V = -d the direction to the eye, L = V for a headlight, else the    */
/* normalised light direction, H = (L + V)/|L + V| (no specular when L = -V) */
/* and n = -g / max(|g|, grad_min): the unit normal where the gradient is  */
/* at least grad_min, shrinking to zero with it below (flat regions get    */
/* ambient light only).  |.| makes the lighting two-sided.  Opacity is      */
/* unchanged.                                                               */
static void or_shade_colour(const double *sh, const double d[3], const double g[3], double c[3])
{
    double V[3] = {-d[0], -d[1], -d[2]}, L[3];
    if (sh[7] != 0.0) {
        for (int a = 0; a < 3; ++a) L[a] = V[a];
    } else {
        double ln = sqrt(sh[4] * sh[4] + sh[5] * sh[5] + sh[6] * sh[6]);
        for (int a = 0; a < 3; ++a) L[a] = sh[4 + a] / ln;
    }
    double Hs[3] = {L[0] + V[0], L[1] + V[1], L[2] + V[2]};
    double hn = sqrt(Hs[0] * Hs[0] + Hs[1] * Hs[1] + Hs[2] * Hs[2]);
    double gm = sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    double m = gm > sh[8] ? gm : sh[8];
    double n[3] = {-g[0] / m, -g[1] / m, -g[2] / m};
    double nl = fabs(n[0] * L[0] + n[1] * L[1] + n[2] * L[2]);
    double spec = 0.0;
    if (hn > 1e-12) {
        double nh = fabs(n[0] * Hs[0] + n[1] * Hs[1] + n[2] * Hs[2]) / hn;
        spec = pow(nh, sh[3]);
    }
    for (int a = 0; a < 3; ++a) c[a] = c[a] * (sh[0] + sh[1] * nl) + sh[2] * spec;
}

/* T at node coordinate u in [0, K-1]: linear between nodes j = min(floor u, */
/* K-2) and j+1 with weight w = u - j.                                       */
static void or_tf_at(const float *tf, int K, double u, double out[4], long *j_out, double *w_out)
{
    long j = (long)floor(u);
    if (j > K - 2) j = K - 2;
    double w = u - (double)j;
    for (int c = 0; c < 4; ++c) out[c] = (1.0 - w) * (double)tf[4 * j + c] + w * (double)tf[4 * (j + 1) + c];
    *j_out = j;
    *w_out = w;
}

/* Post-classification: T(V) on the interpolated value.  Node j sits at      */
/* v0 + j (v1 - v0)/(K-1); u is clamped to [0, K-1]; linear between nodes.   */
/* Outputs (r, g, b, sigma), the segment j, its weight w and whether u was   */
/* clamped.                                                                  */
static void or_classify(const float *tf, int K, double v0, double v1, double v, double out[4], long *j_out,
                        double *w_out, int *clamped)
{
    double u = (v - v0) * (double)(K - 1) / (v1 - v0);
    *clamped = 0;
    if (u < 0.0) {
        u = 0.0;
        *clamped = 1;
    }
    if (u > (double)(K - 1)) {
        u = (double)(K - 1);
        *clamped = 1;
    }
    or_tf_at(tf, K, u, out, j_out, w_out);
}

/* Pre-classification (the alternative the paper weighs against interpolating */
/* first, Section 2, Fig. 4 discussion): every tap is classified, then the   */
/* B-spline interpolates the opacity-weighted channels (sigma r, sigma g,    */
/* sigma b, sigma); the sample's colour is the weighted colour over its      */
/* extinction (0 where the extinction is 0).                                 */
static void or_preclassify(const or_vol *vol, const float *tf, int K, double v0, double v1, const double p[3],
                           double out[4])
{
    long ix = (long)floor(p[0]), iy = (long)floor(p[1]), iz = (long)floor(p[2]);
    double wx[4], wy[4], wz[4];
    or_bspline(p[0] - (double)ix, wx);
    or_bspline(p[1] - (double)iy, wy);
    or_bspline(p[2] - (double)iz, wz);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int c = 0; c < 4; ++c)
        for (int b = 0; b < 4; ++b)
            for (int a = 0; a < 4; ++a) {
                long x = or_clampl(ix - 1 + a, 0, vol->nx - 1);
                long y = or_clampl(iy - 1 + b, 0, vol->ny - 1);
                long z = or_clampl(iz - 1 + c, 0, vol->nz - 1);
                double t[4], tw;
                long tj;
                int tc;
                or_classify(tf, K, v0, v1, or_voxel(vol, x, y, z), t, &tj, &tw, &tc);
                double wt = wx[a] * wy[b] * wz[c];
                for (int q = 0; q < 3; ++q) acc[q] += wt * t[3] * t[q];
                acc[3] += wt * t[3];
            }
    for (int q = 0; q < 3; ++q) out[q] = acc[3] > 0.0 ? acc[q] / acc[3] : 0.0;
    out[3] = acc[3];
}

typedef struct {
    const or_vol *vol;
    const double *cams;
    int W, H;
    const float *tf;
    int K;
    double v0, v1, step, ert;
    const uint8_t *occ; /* NULL: no skipping */
    int edge;
    const double *shade; /* NULL: no local lighting */
    int filter;          /* 0 cubic B-spline, 1 Catmull-Rom */
} or_ctx;

/* Sample lattice: the ray moves from its origin (the observer) with the     */
/* fixed step, sampling at t_k = (k + 1/2) step; the samples of a ray are    */
/* every k >= 0 with t_in < t_k < t_out.  Returns their count and the first  */
/* index k0.  Rays of neighbouring pixels thus share sample distances.       */
static long or_lattice(double tin, double tout, double step, long *k0_out)
{
    long k = (long)floor(tin / step - 0.5);
    if (k < 0) k = 0;
    while (k > 0 && ((double)(k - 1) + 0.5) * step > tin) --k;
    while (((double)k + 0.5) * step <= tin) ++k;
    long k0 = k;
    while (((double)k + 0.5) * step < tout) ++k;
    *k0_out = k0;
    return k - k0;
}

static long or_lattice_count(double tin, double tout, double step)
{
    long k0;
    return or_lattice(tin, tout, step, &k0);
}

static int or_block_occupied(const or_ctx *cx, const double p[3])
{
    long cx_ = or_clampl((long)floor(p[0]), 0, cx->vol->nx - 1);
    long cy_ = or_clampl((long)floor(p[1]), 0, cx->vol->ny - 1);
    long cz_ = or_clampl((long)floor(p[2]), 0, cx->vol->nz - 1);
    long nbx = (cx->vol->nx + cx->edge - 1) / cx->edge, nby = (cx->vol->ny + cx->edge - 1) / cx->edge;
    long b = cx_ / cx->edge + nbx * (cy_ / cx->edge + nby * (cz_ / cx->edge));
    return cx->occ[b] != 0;
}

/* One ray, forward.  rgba gets premultiplied (C, 1 - T) over transparent    */
/* black.  counts[0] = lattice samples, counts[1] = evaluated samples.       */
/* flag = 1 when the termination test came within 1e-5 of the threshold.     */
static void or_trace(const or_ctx *cx, long view, long row, long col, double rgba[4], long counts[2], uint8_t *flag)
{
    double o[3], d[3], tin, tout;
    rgba[0] = rgba[1] = rgba[2] = rgba[3] = 0.0;
    counts[0] = counts[1] = 0;
    *flag = 0;
    const double *cam = cx->cams + 16 * view;
    or_ray(cam, cx->W, cx->H, col, row, o, d);
    if (!or_clip(o, d, cx->vol->nx, cx->vol->ny, cx->vol->nz, &tin, &tout)) return;
    long k0;
    long ns = or_lattice(tin, tout, cx->step, &k0);
    counts[0] = ns;
    int ert_on = cx->ert > 0.0 && cx->ert < 1.0;
    double C[3] = {0.0, 0.0, 0.0}, T = 1.0;
    or_sample s;
    for (long k = k0; k < k0 + ns; ++k) {
        double t = ((double)k + 0.5) * cx->step;
        double p[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
        if (cx->occ && !or_block_occupied(cx, p)) continue;
        counts[1]++;
        double val[4], w;
        long j;
        int cl;
        if (cx->filter == 2) {
            or_preclassify(cx->vol, cx->tf, cx->K, cx->v0, cx->v1, p, val);
        } else {
            or_reconstruct_f(cx->vol, p, &s, cx->filter);
            or_classify(cx->tf, cx->K, cx->v0, cx->v1, s.v, val, &j, &w, &cl);
        }
        if (cx->shade) {
            double g[3];
            or_gradient(cx->vol, p, g);
            or_shade_colour(cx->shade, d, g, val);
        }
        double alpha = -expm1(-val[3] * cx->step);
        for (int c = 0; c < 3; ++c) C[c] += T * alpha * val[c];
        T *= exp(-val[3] * cx->step);
        if (ert_on) {
            if (fabs((1.0 - T) - cx->ert) < 1e-5) *flag = 1;
            if (1.0 - T >= cx->ert) break;
        }
    }
    rgba[0] = C[0];
    rgba[1] = C[1];
    rgba[2] = C[2];
    rgba[3] = 1.0 - T;
}

/* ------------------------------------------------------------------------ */
/* Forward render.                                                           */
/* cams: n_cams x 16 doubles (see or_ray); all views W x H.                  */
/* pix: optional list of n_pix (view, row, col) triples; NULL renders every  */
/* pixel of every view in [view][row][col] order.                            */
/* out_rgba: 4 doubles per output pixel; out_flags (optional): 1 byte;       */
/* out_counts (optional): 2 longs (lattice, evaluated).                      */
/* occ (optional): one byte per block from oracle_occupancy; NULL = no skip. */
/* ------------------------------------------------------------------------ */
static int or_render(const void *data, int dtype, long nx, long ny, long nz, const double *cams, int n_cams, int W,
                     int H, const float *tf, int K, double v0, double v1, double step, double ert,
                     const uint8_t *occ, int edge, const double *shade, int filter, const long *pix, long n_pix,
                     double *out_rgba, uint8_t *out_flags, long *out_counts)
{
    if (!data || !cams || !tf || !out_rgba || n_cams <= 0 || W <= 0 || H <= 0 || K < 2 || !(v1 > v0) ||
        !(step > 0.0))
        return 1;
    if (shade && !(shade[8] > 0.0 && shade[3] >= 1.0)) return 1;
    or_vol vol = {data, dtype, nx, ny, nz};
    if (filter < 0 || filter > 3) return 1;
    or_ctx cx = {&vol, cams, W, H, tf, K, v0, v1, step, ert, occ, edge, shade, filter};
    long total = pix ? n_pix : (long)n_cams * W * H;
#pragma omp parallel for schedule(dynamic, 16)
    for (long q = 0; q < total; ++q) {
        long view, row, col;
        if (pix) {
            view = pix[3 * q];
            row = pix[3 * q + 1];
            col = pix[3 * q + 2];
        } else {
            view = q / ((long)W * H);
            row = (q / W) % H;
            col = q % W;
        }
        double rgba[4];
        long cnt[2];
        uint8_t flag;
        or_trace(&cx, view, row, col, rgba, cnt, &flag);
        for (int c = 0; c < 4; ++c) out_rgba[4 * q + c] = rgba[c];
        if (out_flags) out_flags[q] = flag;
        if (out_counts) {
            out_counts[2 * q] = cnt[0];
            out_counts[2 * q + 1] = cnt[1];
        }
    }
    return 0;
}

/* filter: 0 cubic B-spline (the default reading), 1 Catmull-Rom; occ must */
/* then come from oracle_occupancy with the Catmull-Rom widening.          */
int oracle_render(const void *data, int dtype, long nx, long ny, long nz, const double *cams, int n_cams, int W,
                  int H, const float *tf, int K, double v0, double v1, double step, double ert,
                  const uint8_t *occ, int edge, int filter, const long *pix, long n_pix, double *out_rgba,
                  uint8_t *out_flags, long *out_counts)
{
    return or_render(data, dtype, nx, ny, nz, cams, n_cams, W, H, tf, K, v0, v1, step, ert, occ, edge, NULL, filter,
                     pix, n_pix, out_rgba, out_flags, out_counts);
}

/* Forward render with local lighting; shade as in or_shade_colour.         */
int oracle_render_shaded(const void *data, int dtype, long nx, long ny, long nz, const double *cams, int n_cams,
                         int W, int H, const float *tf, int K, double v0, double v1, double step, double ert,
                         const uint8_t *occ, int edge, const double *shade, const long *pix, long n_pix,
                         double *out_rgba, uint8_t *out_flags, long *out_counts)
{
    if (!shade) return 1;
    return or_render(data, dtype, nx, ny, nz, cams, n_cams, W, H, tf, K, v0, v1, step, ert, occ, edge, shade, 0,
                     pix, n_pix, out_rgba, out_flags, out_counts);
}

/* ------------------------------------------------------------------------ */
/* Gradient of L = sum_pixels <g, RGBA> with respect to the voxel values and */
/* the TF table (the adjoint of the forward model above).                    */
/*                                                                           */
/* Forward: C = sum_k T_k a_k c_k, T_{k+1} = T_k (1 - a_k), A = 1 - T_end,   */
/* a_k = 1 - exp(-s_k step).  Hence                                          */
/*   dC/dc_k     = T_k a_k                                                   */
/*   dC/ds_k     = step (T_{k+1} c_k - S_k),  S_k = sum_{m>k} T_m a_m c_m    */
/*   dA/ds_k     = step T_end                                                */
/* and the chain rule through the TF segment (slope (K-1)/(v1-v0) times the  */
/* node difference, zero where u was clamped) and the 64 B-spline weights.   */
/* The stopping index of early termination is held fixed.  The per-ray      */
/* samples are stored and the suffix sums S_k formed explicitly.             */
/* grad_rgba: 4 doubles per pixel of the full image set.                     */
/* grad_vol (nx*ny*nz) and grad_tf (K*4) are accumulated into (+=).          */
/* mag_vol / mag_tf (optional, same shapes, +=) receive the same sums with  */
/* every term replaced by its magnitude, the suffix-sum difference included */
/* (|T_{k+1} c_k| + |S_k|): the scale of the rounding error of any          */
/* evaluation of these sums, for element-wise error bounds.                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    or_sample s;
    long j;
    double w;
    int clamped;
    double val[4];
    double alpha, Tk;
} or_rec;

int oracle_grad(const void *data, int dtype, long nx, long ny, long nz, const double *cams, int n_cams, int W,
                int H, const float *tf, int K, double v0, double v1, double step, double ert, const uint8_t *occ,
                int edge, const double *grad_rgba, double *grad_vol, double *grad_tf, double *mag_vol,
                double *mag_tf)
{
    if (!data || !cams || !tf || !grad_rgba || n_cams <= 0 || W <= 0 || H <= 0 || K < 2 || !(v1 > v0) ||
        !(step > 0.0))
        return 1;
    or_vol vol = {data, dtype, nx, ny, nz};
    or_ctx cx = {&vol, cams, W, H, tf, K, v0, v1, step, ert, occ, edge, NULL, 0};
    long total = (long)n_cams * W * H;
    double slope_scale = (double)(K - 1) / (v1 - v0);
    int ert_on = ert > 0.0 && ert < 1.0;
#pragma omp parallel
    {
        long cap = 0;
        or_rec *rec = NULL;
#pragma omp for schedule(dynamic, 16)
        for (long q = 0; q < total; ++q) {
            long view = q / ((long)W * H), row = (q / W) % H, col = q % W;
            const double *g = grad_rgba + 4 * q;
            if (g[0] == 0.0 && g[1] == 0.0 && g[2] == 0.0 && g[3] == 0.0) continue;
            double o[3], d[3], tin, tout;
            or_ray(cams + 16 * view, W, H, col, row, o, d);
            if (!or_clip(o, d, nx, ny, nz, &tin, &tout)) continue;
            long k0;
            long ns = or_lattice(tin, tout, step, &k0);
            if (ns > cap) {
                free(rec);
                cap = ns;
                rec = (or_rec *)malloc(sizeof(or_rec) * (size_t)cap);
            }
            /* forward, storing every evaluated sample */
            long n = 0;
            double T = 1.0;
            for (long k = k0; k < k0 + ns; ++k) {
                double t = ((double)k + 0.5) * step;
                double p[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
                if (occ && !or_block_occupied(&cx, p)) continue;
                or_rec *r = &rec[n++];
                or_reconstruct(&vol, p, &r->s);
                or_classify(tf, K, v0, v1, r->s.v, r->val, &r->j, &r->w, &r->clamped);
                r->alpha = -expm1(-r->val[3] * step);
                r->Tk = T;
                T *= exp(-r->val[3] * step);
                if (ert_on && 1.0 - T >= ert) break;
            }
            double Tend = T;
            /* backward: walk from the last sample, S holds sum_{m>k} */
            double S[3] = {0.0, 0.0, 0.0};
            for (long m = n - 1; m >= 0; --m) {
                or_rec *r = &rec[m];
                double Tnext = r->Tk * exp(-r->val[3] * step);
                double dval[4], dmag[4];
                double ds = 0.0, dsmag = 0.0;
                for (int c = 0; c < 3; ++c) {
                    dval[c] = g[c] * r->Tk * r->alpha;
                    ds += g[c] * (Tnext * r->val[c] - S[c]);
                    dmag[c] = fabs(dval[c]);
                    dsmag += fabs(g[c]) * (Tnext * fabs(r->val[c]) + fabs(S[c]));
                }
                ds += g[3] * Tend;
                dsmag += fabs(g[3]) * Tend;
                dval[3] = step * ds;
                dmag[3] = step * dsmag;
                for (int c = 0; c < 3; ++c) S[c] += r->Tk * r->alpha * r->val[c];
                if (grad_tf) {
                    for (int c = 0; c < 4; ++c) {
#pragma omp atomic
                        grad_tf[4 * r->j + c] += (1.0 - r->w) * dval[c];
#pragma omp atomic
                        grad_tf[4 * (r->j + 1) + c] += r->w * dval[c];
                        if (mag_tf) {
#pragma omp atomic
                            mag_tf[4 * r->j + c] += (1.0 - r->w) * dmag[c];
#pragma omp atomic
                            mag_tf[4 * (r->j + 1) + c] += r->w * dmag[c];
                        }
                    }
                }
                if (grad_vol && !r->clamped) {
                    double dv = 0.0, dvmag = 0.0;
                    for (int c = 0; c < 4; ++c) {
                        const double slope =
                            ((double)tf[4 * (r->j + 1) + c] - (double)tf[4 * r->j + c]) * slope_scale;
                        dv += dval[c] * slope;
                        dvmag += dmag[c] * fabs(slope);
                    }
                    for (int t = 0; t < 64; ++t) {
#pragma omp atomic
                        grad_vol[r->s.tap[t]] += dv * r->s.wt[t];
                        if (mag_vol) {
#pragma omp atomic
                            mag_vol[r->s.tap[t]] += dvmag * fabs(r->s.wt[t]);
                        }
                    }
                }
            }
        }
        free(rec);
    }
    return 0;
}

/* Lattice count and ray parameters for one pixel (exposed for tests).       */
int oracle_ray(const double *cam, int W, int H, long row, long col, long nx, long ny, long nz, double step,
               double out[8], long *ns)
{
    double o[3], d[3], tin = 0.0, tout = 0.0;
    or_ray(cam, W, H, col, row, o, d);
    int hit = or_clip(o, d, nx, ny, nz, &tin, &tout);
    for (int k = 0; k < 3; ++k) {
        out[k] = o[k];
        out[3 + k] = d[k];
    }
    out[6] = tin;
    out[7] = tout;
    *ns = hit ? or_lattice_count(tin, tout, step) : 0;
    return hit;
}

/* Tricubic value at an arbitrary point (exposed for the reconstruction pins). */
double oracle_sample(const void *data, int dtype, long nx, long ny, long nz, double px, double py, double pz)
{
    or_vol vol = {data, dtype, nx, ny, nz};
    double p[3] = {px, py, pz};
    or_sample s;
    or_reconstruct(&vol, p, &s);
    return s.v;
}

double oracle_sample_filter(const void *data, int dtype, long nx, long ny, long nz, double px, double py, double pz,
                            int filter)
{
    or_vol vol = {data, dtype, nx, ny, nz};
    double p[3] = {px, py, pz};
    or_sample s;
    or_reconstruct_f(&vol, p, &s, filter);
    return s.v;
}

void oracle_catmull_rom(double f, double w[4]) { or_catmull_rom(f, w); }

/* B-spline weights at fractional offset f (exposed for the weight pins).   */
void oracle_weights(double f, double w[4]) { or_bspline(f, w); }

void oracle_dweights(double f, double d[4]) { or_bspline_deriv(f, d); }

/* Gradient of the reconstructed field at (px, py, pz). */
void oracle_gradient(const void *data, int dtype, long nx, long ny, long nz, double px, double py, double pz,
                     double g[3])
{
    or_vol vol = {data, dtype, nx, ny, nz};
    double p[3] = {px, py, pz};
    or_gradient(&vol, p, g);
}

/* Lattice sample count of every pixel of every view (ray setup and clip     */
/* only; exposed so that integer counts can be compared at full size).       */
int oracle_lattice(const double *cams, int n_cams, int W, int H, long nx, long ny, long nz, double step, long *out)
{
    if (!cams || !out || n_cams <= 0 || W <= 0 || H <= 0 || !(step > 0.0)) return 1;
    long total = (long)n_cams * W * H;
#pragma omp parallel for schedule(static)
    for (long q = 0; q < total; ++q) {
        long view = q / ((long)W * H), row = (q / W) % H, col = q % W;
        double o[3], d[3], tin, tout;
        or_ray(cams + 16 * view, W, H, col, row, o, d);
        out[q] = or_clip(o, d, nx, ny, nz, &tin, &tout) ? or_lattice_count(tin, tout, step) : 0;
    }
    return 0;
}


/* ------------------------------------------------------------------------ */
/* Pre-integrated classification (Section 2: rendering combined with tables */
/* of previously integrated values, and the conclusion's pre-integrated     */
/* rendering against sampling artefacts).                                   */
/*                                                                           */
/* A ray segment of length `step` along which the value rises linearly from */
/* node value i to node value j (u = TF node coordinate) has, with          */
/* u(x) = i + (j - i) x / step, x in [0, step],                             */
/*   tau(x) = integral_0^x sigma(u(x')) dx',                                */
/*   alpha  = 1 - exp(-tau(step)),                                          */
/*   C      = integral_0^step c(u(x)) sigma(u(x)) exp(-tau(x)) dx           */
/* (premultiplied emission of the segment, the emission-absorption model    */
/* integrated exactly along the segment).  The table holds (C, alpha) for   */
/* every node pair.  Quadrature: [0, step] is split where u crosses a node  */
/* (sigma and c are linear between), each piece into sub-intervals of      */
/* optical depth at most 1/256 (at least 16), composite Simpson on each,    */
/* with */
/* tau exact (trapezoid of a linear sigma); integration stops once tau      */
/* exceeds 60 (what follows is below exp(-60)).  i == j: closed form.       */
/* out: K*K*4 doubles, entry (i, j) at 4 (i K + j).                          */
/* ------------------------------------------------------------------------ */
static void or_tf_node_lerp(const float *tf, int K, double u, double out[4])
{
    long j;
    double w;
    if (u <= 0.0) u = 0.0;
    if (u >= (double)(K - 1)) u = (double)(K - 1);
    or_tf_at(tf, K, u, out, &j, &w);
}

static void or_preint_entry(const float *tf, int K, long i, long j, double step, double out[4])
{
    out[0] = out[1] = out[2] = out[3] = 0.0;
    if (i == j) {
        double sg = (double)tf[4 * i + 3];
        double a = -expm1(-sg * step);
        for (int c = 0; c < 3; ++c) out[c] = (double)tf[4 * i + c] * a;
        out[3] = a;
        return;
    }
    long n = labs(j - i);
    long dir = j > i ? 1 : -1;
    double piece = step / (double)n;
    double tau = 0.0, C[3] = {0.0, 0.0, 0.0};
    for (long m = 0; m < n && tau <= 60.0; ++m) {
        double ua = (double)(i + dir * m), ub = (double)(i + dir * (m + 1));
        double ea[4], eb[4];
        or_tf_node_lerp(tf, K, ua, ea);
        or_tf_node_lerp(tf, K, ub, eb);
        /* sigma, c linear in x over [0, piece] from ea to eb */
        double tau_piece = 0.5 * (ea[3] + eb[3]) * piece;
        long sub = (long)ceil(tau_piece * 256.0);
        if (sub < 16) sub = 16;
        double h = piece / (double)sub;
        for (long q = 0; q < sub; ++q) {
            double xs[3] = {q * h, (q + 0.5) * h, (q + 1) * h};
            if (tau + ea[3] * xs[0] + 0.5 * (eb[3] - ea[3]) * xs[0] * xs[0] / piece > 60.0) break;
            double f[3];
            for (int r = 0; r < 3; ++r) {
                double w = xs[r] / piece;
                double sg = (1.0 - w) * ea[3] + w * eb[3];
                /* tau at xs[r]: tau at the piece start + integral of the linear sigma */
                double t = tau + ea[3] * xs[r] + 0.5 * (eb[3] - ea[3]) * xs[r] * xs[r] / piece;
                f[r] = sg * exp(-t);
            }
            for (int c = 0; c < 3; ++c) {
                double cc[3];
                for (int r = 0; r < 3; ++r) {
                    double w = xs[r] / piece;
                    cc[r] = ((1.0 - w) * ea[c] + w * eb[c]) * f[r];
                }
                C[c] += h / 6.0 * (cc[0] + 4.0 * cc[1] + cc[2]);
            }
        }
        tau += tau_piece;
    }
    for (int c = 0; c < 3; ++c) out[c] = C[c];
    out[3] = -expm1(-tau);
}

int oracle_preint_table(const float *tf, int K, double step, double *out)
{
    if (!tf || !out || K < 2 || !(step > 0.0)) return 1;
#pragma omp parallel for schedule(dynamic, 4)
    for (long i = 0; i < K; ++i)
        for (long j = 0; j < K; ++j) or_preint_entry(tf, K, i, j, step, out + 4 * (i * K + j));
    return 0;
}

/* Bilinear lookup of the table at node coordinates (u_f, u_b), each clamped */
/* to [0, K-1] (values beyond the TF range take the end nodes).             */
static void or_preint_lookup(const double *tab, int K, double uf, double ub, double out[4])
{
    double u[2] = {uf, ub}, w[2];
    long n[2];
    for (int a = 0; a < 2; ++a) {
        if (u[a] < 0.0) u[a] = 0.0;
        if (u[a] > (double)(K - 1)) u[a] = (double)(K - 1);
        n[a] = (long)floor(u[a]);
        if (n[a] > K - 2) n[a] = K - 2;
        w[a] = u[a] - (double)n[a];
    }
    for (int c = 0; c < 4; ++c) {
        double p00 = tab[4 * (n[0] * K + n[1]) + c], p10 = tab[4 * ((n[0] + 1) * K + n[1]) + c];
        double p01 = tab[4 * (n[0] * K + n[1] + 1) + c], p11 = tab[4 * ((n[0] + 1) * K + n[1] + 1) + c];
        out[c] = (1.0 - w[0]) * (1.0 - w[1]) * p00 + w[0] * (1.0 - w[1]) * p10 + (1.0 - w[0]) * w[1] * p01 +
                 w[0] * w[1] * p11;
    }
}

/* Block (of the clamped cell of p) for the pre-integrated skip rule. */
static long or_block_index(const or_vol *vol, int edge, const double p[3])
{
    long cx = or_clampl((long)floor(p[0]), 0, vol->nx - 1);
    long cy = or_clampl((long)floor(p[1]), 0, vol->ny - 1);
    long cz = or_clampl((long)floor(p[2]), 0, vol->nz - 1);
    long nbx = (vol->nx + edge - 1) / edge, nby = (vol->ny + edge - 1) / edge;
    return cx / edge + nbx * (cy / edge + nby * (cz / edge));
}

/* ------------------------------------------------------------------------ */
/* Pre-integrated render.  The cells of the lattice (the same cells whose   */
/* midpoints are the post-classified samples, k0 <= k < k0 + ns) are the    */
/* segments: cell k runs from t = k step to (k+1) step, its front value is  */
/* reconstructed at t = k step and its back value at (k+1) step (ns + 1     */
/* values for ns cells; a boundary may lie up to half a step outside the    */
/* box, where clamp-to-edge defines the field).  Each cell takes the        */
/* table's (C, alpha) at (u(front), u(back)); front to back C += T C_seg,   */
/* T *= 1 - alpha; termination after the cell whose opacity reaches the     */
/* threshold.  Skipping (minmax given: per-block (min, max), 2 doubles per  */
/* block): a cell is skipped iff no value between the two blocks' ranges    */
/* can meet non-zero extinction (its ramp then integrates to exactly 0).    */
/* tab: K*K*4 doubles from oracle_preint_table for this TF and step.        */
/* counts: lattice cells, evaluated cells.                                  */
/* ------------------------------------------------------------------------ */
int oracle_render_preint(const void *data, int dtype, long nx, long ny, long nz, const double *cams, int n_cams,
                         int W, int H, const float *tf, int K, double v0, double v1, const double *tab, double step,
                         double ert, const double *minmax, int edge, const long *pix, long n_pix, double *out_rgba,
                         uint8_t *out_flags, long *out_counts)
{
    if (!data || !cams || !tf || !tab || !out_rgba || n_cams <= 0 || W <= 0 || H <= 0 || K < 2 || !(v1 > v0) ||
        !(step > 0.0))
        return 1;
    or_vol vol = {data, dtype, nx, ny, nz};
    float scale32 = (float)(K - 1) / ((float)v1 - (float)v0);
    double scale = (double)(K - 1) / (v1 - v0);
    int ert_on = ert > 0.0 && ert < 1.0;
    long total = pix ? n_pix : (long)n_cams * W * H;
#pragma omp parallel for schedule(dynamic, 16)
    for (long q = 0; q < total; ++q) {
        long view, row, col;
        if (pix) {
            view = pix[3 * q];
            row = pix[3 * q + 1];
            col = pix[3 * q + 2];
        } else {
            view = q / ((long)W * H);
            row = (q / W) % H;
            col = q % W;
        }
        double o[3], d[3], tin, tout, C[3] = {0.0, 0.0, 0.0}, T = 1.0;
        long ns = 0, nev = 0;
        uint8_t flag = 0;
        or_ray(cams + 16 * view, W, H, col, row, o, d);
        if (or_clip(o, d, nx, ny, nz, &tin, &tout)) {
            long k0;
            ns = or_lattice(tin, tout, step, &k0);
            for (long k = k0; k < k0 + ns; ++k) {
                double tf_ = (double)k * step, tb = (double)(k + 1) * step;
                double pf[3] = {o[0] + tf_ * d[0], o[1] + tf_ * d[1], o[2] + tf_ * d[2]};
                double pb[3] = {o[0] + tb * d[0], o[1] + tb * d[1], o[2] + tb * d[2]};
                if (minmax) {
                    long bf = or_block_index(&vol, edge, pf), bb = or_block_index(&vol, edge, pb);
                    double lo = fmin(minmax[2 * bf], minmax[2 * bb]), hi = fmax(minmax[2 * bf + 1], minmax[2 * bb + 1]);
                    if (!or_range_occupied(tf, K, (float)v0, scale32, (float)lo, (float)hi)) continue;
                }
                ++nev;
                or_sample sf, sb;
                or_reconstruct(&vol, pf, &sf);
                or_reconstruct(&vol, pb, &sb);
                double seg[4];
                or_preint_lookup(tab, K, (sf.v - v0) * scale, (sb.v - v0) * scale, seg);
                for (int c = 0; c < 3; ++c) C[c] += T * seg[c];
                T *= 1.0 - seg[3];
                if (ert_on) {
                    if (fabs((1.0 - T) - ert) < 1e-5) flag = 1;
                    if (1.0 - T >= ert) break;
                }
            }
        }
        out_rgba[4 * q] = C[0];
        out_rgba[4 * q + 1] = C[1];
        out_rgba[4 * q + 2] = C[2];
        out_rgba[4 * q + 3] = 1.0 - T;
        if (out_flags) out_flags[q] = flag;
        if (out_counts) {
            out_counts[2 * q] = ns;
            out_counts[2 * q + 1] = nev;
        }
    }
    return 0;
}


/* ------------------------------------------------------------------------ */
/* Interpolating cubic B-spline (the prefiltered spline of the paper's      */
/* filter comparison, Fig. 4 discussion): coefficients c such that the      */
/* B-spline reconstruction with clamp-to-edge addressing passes through     */
/* every voxel value.  Per axis line the condition is                       */
/*   (c[i-1] + 4 c[i] + c[i+1]) / 6 = v[i],  c[-1] = c[0], c[n] = c[n-1],   */
/* a tridiagonal system (diagonal 5 in the first and last rows, for n >= 2; */
/* c = v for n = 1), solved along x, then y, then z (the tensor-product     */
/* condition separates), each line by plain Gaussian elimination of the     */
/* tridiagonal matrix.  out: nx*ny*nz doubles, layout of the volume.        */
/* ------------------------------------------------------------------------ */
static void or_tridiag_line(double *x, long n, long stride, double *sub, double *diag, double *sup, double *rhs)
{
    if (n == 1) return;
    for (long i = 0; i < n; ++i) {
        sub[i] = i > 0 ? 1.0 : 0.0;
        sup[i] = i < n - 1 ? 1.0 : 0.0;
        diag[i] = (i == 0 || i == n - 1) ? 5.0 : 4.0;
        rhs[i] = 6.0 * x[i * stride];
    }
    for (long i = 1; i < n; ++i) {
        double m = sub[i] / diag[i - 1];
        diag[i] -= m * sup[i - 1];
        rhs[i] -= m * rhs[i - 1];
    }
    x[(n - 1) * stride] = rhs[n - 1] / diag[n - 1];
    for (long i = n - 2; i >= 0; --i) x[i * stride] = (rhs[i] - sup[i] * x[(i + 1) * stride]) / diag[i];
}

int oracle_prefilter(const void *data, int dtype, long nx, long ny, long nz, double *out)
{
    if (!data || !out || nx <= 0 || ny <= 0 || nz <= 0) return 1;
    or_vol vol = {data, dtype, nx, ny, nz};
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y)
            for (long x = 0; x < nx; ++x) out[x + nx * (y + ny * z)] = or_voxel(&vol, x, y, z);
    long nmax = nx > ny ? nx : ny;
    if (nz > nmax) nmax = nz;
    double *work = (double *)malloc(sizeof(double) * 4 * (size_t)nmax);
    if (!work) return 1;
    double *sub = work, *diag = work + nmax, *sup = work + 2 * nmax, *rhs = work + 3 * nmax;
    for (long z = 0; z < nz; ++z)
        for (long y = 0; y < ny; ++y) or_tridiag_line(out + nx * (y + ny * z), nx, 1, sub, diag, sup, rhs);
    for (long z = 0; z < nz; ++z)
        for (long x = 0; x < nx; ++x) or_tridiag_line(out + x + nx * ny * z, ny, nx, sub, diag, sup, rhs);
    for (long y = 0; y < ny; ++y)
        for (long x = 0; x < nx; ++x) or_tridiag_line(out + x + nx * y, nz, nx * ny, sub, diag, sup, rhs);
    free(work);
    return 0;
}
