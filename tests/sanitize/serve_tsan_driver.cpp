// The serving scheduler's host threads under ThreadSanitizer, with a CPU
// stand-in for the device: memory is host memory, copies are memcpy, an event
// reports "not ready" for a few queries after it is recorded (work in
// flight), and a batch launch writes into every pixel of its work items the
// request's signature (the v0 of its TF).  Client threads submit, wait (some
// with zero time-outs), check that every pixel of their image carries their
// own signature, and release; another thread reads and resets statistics and
// registers and removes volumes; the server is destroyed with requests still
// queued.  Exits 0 when every image was right.
#include <atomic>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <thread>
#include <vector>

#include "vr.h"
#include "vr_internal.h"

using namespace vr;

namespace {

struct FakeEvent {
  std::atomic<int> remaining{0};
};
std::atomic<unsigned> g_seed{12345};
std::atomic<long> g_items{0};

int small_random() {
  unsigned x = g_seed.fetch_add(2654435761u);
  x ^= x >> 13;
  return (int)(x % 4);
}

hipError_t f_device_count(int *n) {
  *n = 1;
  return hipSuccess;
}
hipError_t f_set_device(int) { return hipSuccess; }
hipError_t f_stream_create(hipStream_t *s) {
  *s = reinterpret_cast<hipStream_t>(new int(0));
  return hipSuccess;
}
hipError_t f_stream_destroy(hipStream_t s) {
  delete reinterpret_cast<int *>(s);
  return hipSuccess;
}
hipError_t f_stream_sync(hipStream_t) { return hipSuccess; }
hipError_t f_event_create(hipEvent_t *e) {
  *e = reinterpret_cast<hipEvent_t>(new FakeEvent());
  return hipSuccess;
}
hipError_t f_event_destroy(hipEvent_t e) {
  delete reinterpret_cast<FakeEvent *>(e);
  return hipSuccess;
}
hipError_t f_event_record(hipEvent_t e, hipStream_t) {
  reinterpret_cast<FakeEvent *>(e)->remaining.store(small_random());
  return hipSuccess;
}
hipError_t f_event_query(hipEvent_t e) {
  FakeEvent *f = reinterpret_cast<FakeEvent *>(e);
  if (f->remaining.load() > 0) {
    f->remaining.fetch_sub(1);
    return hipErrorNotReady;
  }
  return hipSuccess;
}
hipError_t f_stream_wait(hipStream_t, hipEvent_t) { return hipSuccess; }
hipError_t f_alloc(void **p, size_t n) {
  *p = std::malloc(n ? n : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t f_free(void *p) {
  std::free(p);
  return hipSuccess;
}
hipError_t f_copy(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t) {
  std::memcpy(d, s, n);
  return hipSuccess;
}
hipError_t f_occupancy(const VolConst &v, const TfConst &, uint32_t *bits, bool, hipStream_t) {
  std::memset(bits, 0xff, occupancy_bytes(v));
  return hipSuccess;
}
hipError_t f_launch(const ServeSlot *slots, const ServeItem *items, int32_t n, int32_t, unsigned long long *samples,
                    hipStream_t) {
  for (int32_t i = 0; i < n; ++i) {
    const ServeSlot &sl = slots[items[i].slot];
    for (int y = items[i].sy * kSuperEdge; y < (items[i].sy + 1) * kSuperEdge && y < sl.cam.H; ++y)
      for (int x = items[i].sx * kSuperEdge; x < (items[i].sx + 1) * kSuperEdge && x < sl.cam.W; ++x)
        for (int c = 0; c < 4; ++c) sl.out[((size_t)y * sl.cam.W + x) * 4 + c] = sl.tf.v0;
    *samples += kSuperEdge * kSuperEdge;
  }
  g_items.fetch_add(n);
  return hipSuccess;
}
vr_status f_build_blocks(const vr_volume *vol, int32_t edge, vr_blocks **out, VolConst *vc) {
  vr_status st = check_volume(vol, vc);
  if (st) return st;
  vc->nbx = (int32_t)((vol->nx + edge - 1) / edge);
  vc->nby = (int32_t)((vol->ny + edge - 1) / edge);
  vc->nbz = (int32_t)((vol->nz + edge - 1) / edge);
  vc->edge = edge;
  vc->minmax = reinterpret_cast<const float2 *>(vol->data);  // non-null: requests skip (never read here)
  *out = reinterpret_cast<vr_blocks *>(new char[1]);
  return VR_OK;
}
void f_free_blocks(vr_blocks *b) { delete[] reinterpret_cast<char *>(b); }

const ServeOps kFake = {f_device_count, f_set_device, f_stream_create, f_stream_destroy, f_stream_sync,
                        f_event_create, f_event_destroy, f_event_record, f_event_query,  f_stream_wait,
                        f_alloc,        f_free,       f_alloc,         f_free,          f_copy,
                        f_occupancy,    f_launch,     f_build_blocks,  f_free_blocks};

alignas(16) int16_t g_voxels[64];
std::atomic<int> g_bad{0};

vr_camera camera(int W, int H, int nx) {
  vr_camera c;
  std::memset(&c, 0, sizeof(c));
  c.projection = 1;
  c.width = W;
  c.height = H;
  const double e[3] = {0.5 * nx, -3.0 * nx, 0.5 * nx}, f[3] = {0, 1, 0}, r[3] = {1, 0, 0}, u[3] = {0, 0, 1};
  for (int a = 0; a < 3; ++a) {
    c.eye[a] = e[a];
    c.forward[a] = f[a];
    c.right[a] = r[a];
    c.up[a] = u[a];
  }
  c.fov_y = 0.8;
  return c;
}

}  // namespace

int main() {
  vr_serve_config cfg{};
  cfg.hbm_budget_bytes = 3 * (80 * 80 * 16) + (3u << 20);
  cfg.max_inflight = 6;
  cfg.max_batch_tiles = 7;
  vr_server *srv = nullptr;
  if (serve_create_with_ops(&cfg, &kFake, &srv) != VR_OK) {
    std::fprintf(stderr, "create: %s\n", vr_last_error());
    return 1;
  }
  std::vector<int32_t> ids;
  for (int k = 0; k < 3; ++k) {
    vr_volume v{g_voxels, VR_I16, 0, 64 + 32 * k, 48, 40};
    int32_t id = -1;
    if (vr_serve_add_volume(srv, &v, 16, &id) != VR_OK) return 2;
    ids.push_back(id);
  }
  alignas(16) static float table[8 * 4];
  std::atomic<int> next_sig{1};
  auto client = [&](int seed) {
    std::mt19937 rng(seed);
    for (int q = 0; q < 60; ++q) {
      const int vid = ids[rng() % ids.size()];
      const int W = 16 + (int)(rng() % 65), H = 16 + (int)(rng() % 65);
      const float sig = (float)next_sig.fetch_add(1);
      vr_request r{};
      r.volume_id = vid;
      r.K = 8;
      r.tf_table_host = table;
      r.tf_v0 = sig;
      r.tf_v1 = sig + 1000.0f;
      r.cam = camera(W, H, 64);
      r.step = 0.5f;
      r.ert_threshold = 0.99f;
      r.use_skip = (int)(rng() % 2);
      uint64_t t = 0;
      if (vr_serve_submit(srv, &r, &t) != VR_OK) {
        g_bad++;
        continue;
      }
      const float *img = nullptr;
      if (rng() % 4 == 0) (void)vr_serve_wait(srv, t, 0, &img);  // may time out
      if (vr_serve_wait(srv, t, -1, &img) != VR_OK) {
        g_bad++;
        continue;
      }
      for (size_t i = 0; i < (size_t)W * H * 4; ++i)
        if (img[i] != sig) {
          g_bad++;
          break;
        }
      if (vr_serve_release(srv, t) != VR_OK) g_bad++;
    }
  };
  std::atomic<bool> stop{false};
  std::thread admin([&] {
    int toggles = 0;
    while (!stop.load()) {
      vr_serve_stats st;
      (void)vr_serve_stats_get(srv, &st);
      if (++toggles % 7 == 0) (void)vr_serve_stats_reset(srv);
      vr_volume v{g_voxels, VR_I16, 0, 32, 32, 32};
      int32_t id = -1;
      if (vr_serve_add_volume(srv, &v, 16, &id) == VR_OK) (void)vr_serve_remove_volume(srv, id);
      std::this_thread::sleep_for(std::chrono::microseconds(200));
    }
  });
  std::vector<std::thread> clients;
  for (int c = 0; c < 4; ++c) clients.emplace_back(client, 100 + c);
  for (auto &th : clients) th.join();
  stop = true;
  admin.join();
  // destroy with requests still queued: their waits end with VR_E_SHUTDOWN
  std::vector<uint64_t> pending;
  for (int q = 0; q < 20; ++q) {
    vr_request r{};
    r.volume_id = ids[0];
    r.K = 8;
    r.tf_table_host = table;
    r.tf_v0 = 1.0f;
    r.tf_v1 = 2.0f;
    r.cam = camera(80, 80, 64);
    r.step = 0.5f;
    uint64_t t = 0;
    if (vr_serve_submit(srv, &r, &t) == VR_OK) pending.push_back(t);
  }
  std::atomic<int> ended{0};
  std::vector<std::thread> waiters;
  for (uint64_t t : pending)
    waiters.emplace_back([&, t] {
      const float *img = nullptr;
      const vr_status st = vr_serve_wait(srv, t, -1, &img);
      if (st == VR_OK || st == VR_E_SHUTDOWN) ended++;
    });
  (void)vr_serve_destroy(srv);
  for (auto &th : waiters) th.join();
  std::printf("serve tsan driver: %s (%d bad, %ld items, %d/%zu waits ended)\n",
              g_bad.load() || ended.load() != (int)pending.size() ? "FAILED" : "ok", g_bad.load(), g_items.load(),
              ended.load(), pending.size());
  return g_bad.load() || ended.load() != (int)pending.size() ? 1 : 0;
}
