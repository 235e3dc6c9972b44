// Host-side paths of the C ABI without a device, for a build of the library's
// host code with AddressSanitizer and UndefinedBehaviorSanitizer: argument
// validation of every entry point (each call must fail with its documented
// status before touching the device) and the host-only brick ordering over
// many cameras and volume shapes.  Exits 0 when every status is as expected.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "vr.h"
#include "vr_probe.h"

static int failures = 0;

static void expect(vr_status got, vr_status want, const char *what) {
  if (got != want) {
    std::fprintf(stderr, "%s: status %d, expected %d (%s)\n", what, (int)got, (int)want, vr_last_error());
    ++failures;
  }
}

static vr_camera make_cam(int proj, double ex, double ey, double ez, double fx, double fy, double fz, int W, int H) {
  vr_camera c;
  std::memset(&c, 0, sizeof(c));
  c.projection = proj;
  c.width = W;
  c.height = H;
  const double n = std::sqrt(fx * fx + fy * fy + fz * fz);
  const double f[3] = {fx / n, fy / n, fz / n};
  double up[3] = {0.0, 0.0, 1.0};
  if (std::fabs(f[2]) > 0.99) {
    up[1] = 1.0;
    up[2] = 0.0;
  }
  double r[3] = {f[1] * up[2] - f[2] * up[1], f[2] * up[0] - f[0] * up[2], f[0] * up[1] - f[1] * up[0]};
  const double rn = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
  for (double &x : r) x /= rn;
  const double u[3] = {r[1] * f[2] - r[2] * f[1], r[2] * f[0] - r[0] * f[2], r[0] * f[1] - r[1] * f[0]};
  const double e[3] = {ex, ey, ez};
  for (int a = 0; a < 3; ++a) {
    c.eye[a] = e[a];
    c.right[a] = r[a];
    c.up[a] = u[a];
    c.forward[a] = f[a];
  }
  c.fov_y = 1.0;
  c.ortho_w = 64.0;
  c.ortho_h = 48.0;
  return c;
}

int main() {
  if (vr_abi_version() != VR_ABI_VERSION) ++failures;
  const vr_status ds = vr_device_status(nullptr);  // no device here: VR_E_DEVICE (VR_OK on a clean device)
  if (ds != VR_E_DEVICE && ds != VR_OK) ++failures;
  // a volume and TF that pass validation (data pointers are never read)
  alignas(16) static float table[16 * 4];
  static int16_t voxels[8];
  vr_volume vol{voxels, VR_I16, 0, 2, 2, 2};
  vr_tf tf{table, 16, -1024.0f, 3056.0f};
  vr_params p{};
  p.step = 0.5f;
  vr_camera cam = make_cam(1, -10, -10, -10, 1, 1, 1, 8, 8);
  float *out = reinterpret_cast<float *>(table);
  vr_blocks *blocks = nullptr;
  // every entry point, each with one invalid argument
  expect(vr_build_blocks(nullptr, 16, nullptr, &blocks), VR_E_INVALID_ARG, "build_blocks null volume");
  expect(vr_build_blocks(&vol, 3, nullptr, &blocks), VR_E_INVALID_ARG, "build_blocks edge");
  expect(vr_build_blocks(&vol, 16, nullptr, nullptr), VR_E_INVALID_ARG, "build_blocks null out");
  vr_volume big = vol;
  big.nx = big.ny = 1 << 15;
  big.nz = 4;
  expect(vr_build_blocks(&big, 16, nullptr, &blocks), VR_E_UNSUPPORTED, "build_blocks 4 GiB");
  vr_volume odd = vol;
  odd.data = reinterpret_cast<const char *>(voxels) + 2;
  expect(vr_render(&odd, nullptr, &cam, 1, &tf, &p, out, nullptr), VR_E_INVALID_ARG, "render misaligned");
  expect(vr_blocks_info(nullptr, nullptr, nullptr), VR_E_INVALID_ARG, "blocks_info");
  expect(vr_blocks_minmax(nullptr, out, 4, nullptr), VR_E_INVALID_ARG, "blocks_minmax");
  expect(vr_block_occupancy(nullptr, &tf, nullptr, 0, nullptr), VR_E_INVALID_ARG, "block_occupancy");
  vr_params bad = p;
  bad.step = 0.0f;
  expect(vr_render(&vol, nullptr, &cam, 1, &tf, &bad, out, nullptr), VR_E_INVALID_ARG, "render step");
  bad = p;
  bad.use_skip = 1;
  expect(vr_render(&vol, nullptr, &cam, 1, &tf, &bad, out, nullptr), VR_E_INVALID_ARG, "render skip no blocks");
  bad = p;
  bad.filter = 9;
  expect(vr_render(&vol, nullptr, &cam, 1, &tf, &bad, out, nullptr), VR_E_INVALID_ARG, "render filter");
  expect(vr_render(&vol, nullptr, nullptr, 0, &tf, &p, out, nullptr), VR_E_INVALID_ARG, "render no cameras");
  expect(vr_render(&vol, nullptr, &cam, 1, &tf, &p, nullptr, nullptr), VR_E_INVALID_ARG, "render null out");
  vr_tf bad_tf = tf;
  bad_tf.K = 1;
  expect(vr_render(&vol, nullptr, &cam, 1, &bad_tf, &p, out, nullptr), VR_E_INVALID_ARG, "render K");
  bad_tf = tf;
  bad_tf.v1 = bad_tf.v0;
  expect(vr_render(&vol, nullptr, &cam, 1, &bad_tf, &p, out, nullptr), VR_E_INVALID_ARG, "render range");
  vr_camera c2 = cam;
  c2.eye[1] = NAN;
  expect(vr_render(&vol, nullptr, &c2, 1, &tf, &p, out, nullptr), VR_E_INVALID_ARG, "render nan camera");
  c2 = cam;
  c2.width = 0;
  expect(vr_render(&vol, nullptr, &c2, 1, &tf, &p, out, nullptr), VR_E_INVALID_ARG, "render width");
  vr_camera two[2] = {cam, cam};
  two[1].height = 9;
  expect(vr_render(&vol, nullptr, two, 2, &tf, &p, out, nullptr), VR_E_INVALID_ARG, "render mixed sizes");
  expect(vr_render_noalloc(&vol, nullptr, &cam, 1, &tf, &bad, out, nullptr), VR_E_INVALID_ARG, "noalloc filter");
  expect(vr_render_shaded(&vol, nullptr, &cam, 1, &tf, &p, nullptr, out, nullptr), VR_E_INVALID_ARG, "shaded null");
  vr_shading sh{};
  sh.ambient = 0.3f;
  sh.shininess = 0.5f;
  sh.grad_min = 1.0f;
  sh.headlight = 1;
  expect(vr_render_shaded(&vol, nullptr, &cam, 1, &tf, &p, &sh, out, nullptr), VR_E_INVALID_ARG, "shininess");
  vr_preint *pre = nullptr;
  expect(vr_preint_build(&bad_tf, 0.5f, nullptr, &pre), VR_E_INVALID_ARG, "preint range");
  expect(vr_render_preint(&vol, nullptr, &cam, 1, &tf, &p, nullptr, out, nullptr), VR_E_INVALID_ARG, "preint null");
  expect(vr_prefilter_bspline(&vol, nullptr, nullptr), VR_E_INVALID_ARG, "prefilter null");
  expect(vr_render_backward(&vol, nullptr, &cam, 1, &tf, &p, nullptr, nullptr, nullptr, nullptr, nullptr),
         VR_E_INVALID_ARG, "backward null");
  vr_bricked *bv = nullptr;
  expect(vr_bricked_create(&vol, 12, 1 << 20, &bv), VR_E_INVALID_ARG, "bricked edge");
  expect(vr_bricked_create(nullptr, 16, 1 << 20, &bv), VR_E_INVALID_ARG, "bricked null");
  expect(vr_bricked_render(nullptr, &cam, 1, &tf, &p, out, nullptr), VR_E_INVALID_ARG, "bricked render null");
  expect(vr_bricked_stats_get(nullptr, nullptr), VR_E_INVALID_ARG, "bricked stats");
  vr_serve_config cfg{};
  cfg.hbm_budget_bytes = 0;
  cfg.max_inflight = 4;
  vr_server *srv = nullptr;
  expect(vr_serve_create(&cfg, &srv), VR_E_INVALID_ARG, "serve budget");
  cfg.hbm_budget_bytes = 1 << 20;
  cfg.max_inflight = 0;
  expect(vr_serve_create(&cfg, &srv), VR_E_INVALID_ARG, "serve slots");
  expect(vr_serve_submit(nullptr, nullptr, nullptr), VR_E_INVALID_ARG, "serve submit");
  expect(vr_serve_wait(nullptr, 1, 0, nullptr), VR_E_INVALID_ARG, "serve wait");
  expect(vr_serve_release(nullptr, 1), VR_E_INVALID_ARG, "serve release");
  expect(vr_serve_stats_get(nullptr, nullptr), VR_E_INVALID_ARG, "serve stats");
  expect(vr_serve_stats_reset(nullptr), VR_E_INVALID_ARG, "serve reset");
  expect(vr_serve_add_volume(nullptr, &vol, 16, nullptr), VR_E_INVALID_ARG, "serve add");
  expect(vr_serve_add_host_volume(nullptr, &vol, 64, nullptr), VR_E_INVALID_ARG, "serve add host");
  expect(vr_serve_remove_volume(nullptr, 0), VR_E_INVALID_ARG, "serve remove");
  expect(vr_serve_destroy(nullptr), VR_E_INVALID_ARG, "serve destroy");
  expect(vr_probe_stream_read(nullptr, 16, nullptr, nullptr), VR_E_INVALID_ARG, "probe null");
  expect(vr_probe_stream_read(table, 15, reinterpret_cast<uint32_t *>(table), nullptr), VR_E_INVALID_ARG,
         "probe size");
  // host-only: brick order for many cameras and shapes; every brick once
  const int64_t shapes[4][3] = {{1, 1, 1}, {96, 80, 72}, {37, 290, 23}, {512, 512, 5382}};
  for (const auto &d : shapes)
    for (int edge : {8, 16, 64}) {
      const int64_t nb = ((d[0] + edge - 1) / edge) * ((d[1] + edge - 1) / edge) * ((d[2] + edge - 1) / edge);
      std::vector<int64_t> order((size_t)nb);
      for (int k = 0; k < 6; ++k) {
        const double t = 0.7 * k;
        vr_camera c = make_cam(k % 2, d[0] * (0.5 + std::cos(t)), d[1] * (0.5 + std::sin(t)), d[2] * 1.5,
                               -std::cos(t), -std::sin(t), -0.6 - 0.1 * k, 16, 16);
        expect(vr_brick_order(d, edge, &c, order.data(), nb), VR_OK, "brick order");
        std::vector<char> seen((size_t)nb, 0);
        for (int64_t b : order) {
          if (b < 0 || b >= nb || seen[(size_t)b]) ++failures;
          else seen[(size_t)b] = 1;
        }
      }
      expect(vr_brick_order(d, edge, &cam, order.data(), nb - 1), VR_E_INVALID_ARG, "brick order short");
    }
  if (std::strlen(vr_last_error()) == 0) ++failures;
  std::printf("abi driver: %s (%d failures)\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
