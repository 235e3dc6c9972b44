/* Exercise every entry point of the C oracle on small seeded inputs, edge
 * cases included (one-voxel and thin volumes, every dtype, cameras inside
 * the volume and on a face, pixel lists, the smallest and largest tables),
 * for a build with AddressSanitizer and UndefinedBehaviorSanitizer.  Exits 0
 * when every call accepted its arguments; the sanitizers abort otherwise. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_num_threads(void);
void oracle_set_num_threads(int n);
int oracle_blocks(const void *data, int dtype, long nx, long ny, long nz, int edge, double *out);
int oracle_occupancy(const double *minmax, long nblocks, const float *tf, int K, float v0, float v1, float widen,
                     uint8_t *occ);
int oracle_render(const void *data, int dtype, long nx, long ny, long nz, const double *cams, int n_cams, int W, int H,
                  const float *tf, int K, double v0, double v1, double step, double ert, const uint8_t *occ, int edge,
                  int filter, const long *pix, long n_pix, double *out_rgba, uint8_t *out_flags, long *out_counts);
int oracle_render_shaded(const void *data, int dtype, long nx, long ny, long nz, const double *cams, int n_cams, int W,
                         int H, const float *tf, int K, double v0, double v1, double step, double ert,
                         const uint8_t *occ, int edge, const double *shade, const long *pix, long n_pix,
                         double *out_rgba, uint8_t *out_flags, long *out_counts);
int oracle_grad(const void *data, int dtype, long nx, long ny, long nz, const double *cams, int n_cams, int W, int H,
                const float *tf, int K, double v0, double v1, double step, double ert, const uint8_t *occ, int edge,
                const double *grad_rgba, double *grad_vol, double *grad_tf, double *mag_vol, double *mag_tf);
int oracle_ray(const double *cam, int W, int H, long row, long col, long nx, long ny, long nz, double step,
               double out[8], long *ns);
double oracle_sample(const void *data, int dtype, long nx, long ny, long nz, double px, double py, double pz);
double oracle_sample_filter(const void *data, int dtype, long nx, long ny, long nz, double px, double py, double pz,
                            int filter);
void oracle_catmull_rom(double f, double w[4]);
void oracle_weights(double f, double w[4]);
void oracle_dweights(double f, double d[4]);
void oracle_gradient(const void *data, int dtype, long nx, long ny, long nz, double px, double py, double pz,
                     double g[3]);
int oracle_lattice(const double *cams, int n_cams, int W, int H, long nx, long ny, long nz, double step, long *out);
int oracle_preint_table(const float *tf, int K, double step, double *out);
int oracle_render_preint(const void *data, int dtype, long nx, long ny, long nz, const double *cams, int n_cams, int W,
                         int H, const float *tf, int K, double v0, double v1, const double *tab, double step,
                         double ert, const double *minmax, int edge, const long *pix, long n_pix, double *out_rgba,
                         uint8_t *out_flags, long *out_counts);
int oracle_prefilter(const void *data, int dtype, long nx, long ny, long nz, double *out);

static uint64_t rng = 88172645463325252ull;
static double urand(void) {
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) / 9007199254740992.0;
}

static void fail(const char *what) {
    fprintf(stderr, "oracle rejected: %s\n", what);
    exit(2);
}

/* camera rows: projection, eye, right, up, forward, fov_y, ortho_w, ortho_h */
static void camera(double *c, int persp, const double eye[3], const double fwd[3], double fov, double ow, double oh) {
    double up0[3] = {0.0, 0.0, 1.0};
    if (fabs(fwd[2]) > 0.99) {
        up0[1] = 1.0;
        up0[2] = 0.0;
    }
    double r[3] = {fwd[1] * up0[2] - fwd[2] * up0[1], fwd[2] * up0[0] - fwd[0] * up0[2],
                   fwd[0] * up0[1] - fwd[1] * up0[0]};
    double n = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    for (int a = 0; a < 3; ++a) r[a] /= n;
    double u[3] = {r[1] * fwd[2] - r[2] * fwd[1], r[2] * fwd[0] - r[0] * fwd[2], r[0] * fwd[1] - r[1] * fwd[0]};
    c[0] = persp;
    for (int a = 0; a < 3; ++a) {
        c[1 + a] = eye[a];
        c[4 + a] = r[a];
        c[7 + a] = u[a];
        c[10 + a] = fwd[a];
    }
    c[13] = fov;
    c[14] = ow;
    c[15] = oh;
}

static void run_volume(long nx, long ny, long nz, int dtype) {
    const long n = nx * ny * nz;
    const size_t esz = dtype == 0 || dtype == 1 ? 2 : (dtype == 2 ? 4 : 8);
    void *vol = malloc((size_t)n * esz);
    for (long i = 0; i < n; ++i) {
        double v = urand() < 0.4 ? 0.0 : 3000.0 * urand();
        if (dtype == 0) ((uint16_t *)vol)[i] = (uint16_t)v;
        else if (dtype == 1) ((int16_t *)vol)[i] = (int16_t)(v - 1000.0);
        else if (dtype == 2) ((float *)vol)[i] = (float)v;
        else ((double *)vol)[i] = v;
    }
    const int Ks[3] = {2, 16, 1024};
    const double v0 = dtype == 1 ? -1024.0 : 0.0, v1 = v0 + 4080.0;
    double cams[16 * 4];
    const double c0[3] = {0.5 * (nx - 1), 0.5 * (ny - 1), 0.5 * (nz - 1)};
    const double dir[3] = {0.36, -0.48, 0.8};
    const double eye0[3] = {c0[0] - 3.0 * (nx + ny + nz) * dir[0], c0[1] - 3.0 * (nx + ny + nz) * dir[1],
                            c0[2] - 3.0 * (nx + ny + nz) * dir[2]};
    camera(cams, 1, eye0, dir, 0.9, 0.0, 0.0);
    const double zf[3] = {0.0, 0.0, 1.0};
    const double eye1[3] = {c0[0], c0[1], -50.0};
    camera(cams + 16, 0, eye1, zf, 0.0, (double)nx + 2.0, (double)ny + 2.0);
    camera(cams + 32, 1, c0, dir, 1.4, 0.0, 0.0); /* inside the volume */
    const double face[3] = {c0[0], c0[1], -0.5};
    camera(cams + 48, 1, face, zf, 1.2, 0.0, 0.0); /* on a face */
    const int W = 9, H = 7, V = 4;
    const long npix = (long)V * W * H;
    double *rgba = malloc(sizeof(double) * 4 * (size_t)npix);
    uint8_t *flags = malloc((size_t)npix);
    long *counts = malloc(sizeof(long) * 2 * (size_t)npix);
    const int edge = 4;
    const long nb = ((nx + edge - 1) / edge) * ((ny + edge - 1) / edge) * ((nz + edge - 1) / edge);
    double *mm = malloc(sizeof(double) * 2 * (size_t)nb);
    uint8_t *occ = malloc((size_t)nb);
    if (oracle_blocks(vol, dtype, nx, ny, nz, edge, mm)) fail("blocks");
    for (int ki = 0; ki < 3; ++ki) {
        const int K = Ks[ki];
        float *tf = malloc(sizeof(float) * 4 * (size_t)K);
        for (int j = 0; j < K; ++j) {
            for (int c = 0; c < 3; ++c) tf[4 * j + c] = (float)urand();
            tf[4 * j + 3] = j < K / 4 ? 0.0f : (float)(0.05 * urand());
        }
        if (oracle_occupancy(mm, nb, tf, K, (float)v0, (float)v1, 0.0f, occ)) fail("occupancy");
        for (int filter = 0; filter < 4; ++filter)
            if (oracle_render(vol, dtype, nx, ny, nz, cams, V, W, H, tf, K, v0, v1, 0.37, 0.99, filter == 1 ? NULL : occ,
                              edge, filter, NULL, npix, rgba, flags, counts))
                fail("render");
        long pix[3 * 5] = {0, 0, 0, 1, H - 1, W - 1, 2, 3, 4, 3, 0, W - 1, 3, H - 1, 0};
        if (oracle_render(vol, dtype, nx, ny, nz, cams, V, W, H, tf, K, v0, v1, 0.5, 0.0, NULL, edge, 0, pix, 5, rgba,
                          flags, counts))
            fail("render pixels");
        const double shade[9] = {0.3, 0.6, 0.4, 12.0, 0.5, -0.5, -0.7, 0.0, 5.0};
        if (oracle_render_shaded(vol, dtype, nx, ny, nz, cams, V, W, H, tf, K, v0, v1, 0.5, 0.9, occ, edge, shade,
                                 NULL, npix, rgba, flags, counts))
            fail("render shaded");
        double *g = malloc(sizeof(double) * 4 * (size_t)npix);
        for (long i = 0; i < 4 * npix; ++i) g[i] = urand() - 0.5;
        double *gv = calloc((size_t)n, sizeof(double)), *mv = calloc((size_t)n, sizeof(double));
        double *gt = calloc((size_t)K * 4, sizeof(double)), *mt = calloc((size_t)K * 4, sizeof(double));
        if (oracle_grad(vol, dtype, nx, ny, nz, cams, V, W, H, tf, K, v0, v1, 0.5, 0.8, NULL, edge, g, gv, gt, mv, mt))
            fail("grad");
        if (oracle_grad(vol, dtype, nx, ny, nz, cams, V, W, H, tf, K, v0, v1, 0.5, 0.0, occ, edge, g, gv, NULL, NULL,
                        NULL))
            fail("grad volume only");
        if (K <= 16) {
            double *tab = malloc(sizeof(double) * 4 * (size_t)K * (size_t)K);
            if (oracle_preint_table(tf, K, 0.5, tab)) fail("preint table");
            if (oracle_render_preint(vol, dtype, nx, ny, nz, cams, V, W, H, tf, K, v0, v1, tab, 0.5, 0.99, mm, edge,
                                     NULL, npix, rgba, flags, counts))
                fail("render preint");
            free(tab);
        }
        free(g);
        free(gv);
        free(mv);
        free(gt);
        free(mt);
        free(tf);
    }
    double *coef = malloc(sizeof(double) * (size_t)n);
    if (oracle_prefilter(vol, dtype, nx, ny, nz, coef)) fail("prefilter");
    long *lat = malloc(sizeof(long) * (size_t)npix);
    if (oracle_lattice(cams, V, W, H, nx, ny, nz, 0.3, lat)) fail("lattice");
    double out8[8];
    long ns = 0;
    (void)oracle_ray(cams, W, H, 3, 4, nx, ny, nz, 0.5, out8, &ns);
    double w[4], grad[3];
    for (int i = 0; i < 20; ++i) {
        const double p[3] = {urand() * (nx + 2) - 1.5, urand() * (ny + 2) - 1.5, urand() * (nz + 2) - 1.5};
        (void)oracle_sample(vol, dtype, nx, ny, nz, p[0], p[1], p[2]);
        for (int f = 1; f < 4; ++f) (void)oracle_sample_filter(vol, dtype, nx, ny, nz, p[0], p[1], p[2], f);
        oracle_gradient(vol, dtype, nx, ny, nz, p[0], p[1], p[2], grad);
        oracle_weights(p[0] - floor(p[0]), w);
        oracle_dweights(p[0] - floor(p[0]), w);
        oracle_catmull_rom(p[0] - floor(p[0]), w);
    }
    free(lat);
    free(coef);
    free(mm);
    free(occ);
    free(rgba);
    free(flags);
    free(counts);
    free(vol);
}

int main(void) {
    oracle_set_num_threads(2);
    if (oracle_num_threads() != 2) fail("threads");
    const long dims[6][3] = {{1, 1, 1}, {2, 3, 4}, {5, 1, 7}, {37, 29, 23}, {16, 16, 16}, {9, 40, 3}};
    for (int d = 0; d < 6; ++d)
        for (int dt = 0; dt < 4; ++dt) run_volume(dims[d][0], dims[d][1], dims[d][2], dt);
    printf("oracle driver: ok\n");
    return 0;
}
