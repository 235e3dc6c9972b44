// serve.cpp -- continuous-batching render server behind vr_serve_*.
//
// The paper serves many clients from one rendering application in the cloud
// (Section 2, "Cloud architecture": several clients share one application;
// Section 3: interactive rendering of a large CT for remote clients).  Here
// volumes and their block structures stay resident in HBM; clients submit
// requests (volume, camera, TF, step) from any thread; a scheduler thread
//   1. admits queued requests in FIFO order while a slot is free and the
//      request's device memory (result image, occupancy buffer) fits the HBM
//      budget next to the resident volumes and their blocks,
//   2. cuts every admitted request into 16x16-pixel work items and fills each
//      launch round-robin from all admitted requests (so requests of
//      different volumes, image sizes and TFs share launches, and a request
//      that arrives while others are on the GPU joins the next launch),
//   3. keeps two launches in flight on two streams, each launch carrying its
//      own copy of the request descriptors and TF tables (no cross-stream
//      dependencies), and retires requests when their last item completes;
//   4. hands admitted requests on out-of-core volumes (host bricks, the
//      paper's block decomposition of data beyond GPU memory) to a worker
//      thread that renders them one at a time through the shared brick pool,
//      pass by pass on a third stream, while in-core requests keep batching.
// The per-pixel arithmetic is the whole-image kernel's, so a request's image
// is the same alone and in any mix.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "vr.h"
#include "vr_internal.h"

using namespace vr;

namespace {

using Clock = std::chrono::steady_clock;

double now_s() { return std::chrono::duration<double>(Clock::now().time_since_epoch()).count(); }

enum class RState { Queued, Admitted, Done, Cancelled, Failed };

struct Request {
  uint64_t ticket = 0;
  int32_t volume_id = 0;
  CamConst cam{};
  vr_camera cam_desc{};     // as submitted (the out-of-core path takes it)
  bool out_of_core = false;
  std::vector<float> tf;  // K*4, host copy
  int32_t K = 0;
  float v0 = 0, v1 = 1;
  MarchConst mc{};
  RState state = RState::Queued;
  vr_status error = VR_OK;
  double t_submit = 0, t_done = 0;
  float *image = nullptr;
  size_t image_bytes = 0;
  int64_t items_total = 0, items_issued = 0, items_done = 0;
  int32_t stx = 0, sty = 0;  // super-tile grid
  std::vector<int32_t> order;  // super-tiles, nearest to the projected volume centre first
  bool released = false;
  // block occupancy under this request's TF and the radius plane (the
  // kernels' cheap leaps), computed by the first batch that carries it
  uint32_t *occ = nullptr;
  size_t occ_bytes = 0;
  int32_t occ_radius = 0;
  int occ_batch = -1;      // batch that computed it
  uint64_t occ_gen = 0;    // that batch's issue generation
};

struct Volume {
  vr_volume desc{};
  VolConst vc{};
  bool radius_fits = false;  // the radius plane can be built for its block grid
  vr_blocks *blocks = nullptr;
  vr_bricked *bricked = nullptr;  // out of core: host bricks (no device volume, no blocks)
  size_t resident_bytes = 0;  // the volume's memory + its blocks, or its bricked structures (charged)
  int64_t users = 0;  // queued + admitted requests
};

// A launch in flight.  Device layout of `dev`: ServeSlot[n_slots], then the
// TF tables (K_i * 4 floats each, 16-byte aligned), then ServeItem[n_items].
struct Batch {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  hipEvent_t occ_done = nullptr;  // after the occupancy launches of this batch
  uint64_t gen = 0;               // issue generation
  char *host = nullptr;  // pinned staging
  char *dev = nullptr;
  size_t cap = 0;
  bool busy = false;
  std::vector<std::pair<uint64_t, int32_t>> per_request;  // ticket, items in this batch
  int64_t pixels = 0;
  unsigned long long *samples_host = nullptr;  // pinned: the launch's evaluated samples, copied after it
};

size_t align16(size_t x) { return (x + 15) & ~size_t(15); }

}  // namespace

struct vr_server {
  vr_serve_config cfg{};
  const ServeOps *ops = nullptr;  // device operations (HIP, or a CPU stand-in)
  std::mutex mu;
  std::condition_variable cv_work;   // scheduler wake-up
  std::condition_variable cv_done;   // waiters
  std::thread thread;
  bool stop = false;
  bool dead = false;
  int waiters = 0;                   // threads inside vr_serve_wait
  vr_status dead_status = VR_OK;

  std::map<int32_t, Volume> volumes;
  int32_t next_volume = 0;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> requests;
  std::deque<uint64_t> queue;         // FIFO of queued tickets
  std::vector<uint64_t> admitted;     // tickets holding a slot
  uint64_t next_ticket = 1;
  size_t rr = 0;                      // round-robin cursor over admitted

  // HBM accounting: resident volumes and blocks, result images, occupancy
  // buffers (pooled ones included until they are evicted)
  uint64_t hbm_used = 0, hbm_peak = 0;
  uint64_t resident_bytes = 0;  // volumes + blocks
  std::multimap<size_t, float *> image_pool;  // free images by size
  std::multimap<size_t, uint32_t *> occ_pool;  // free occupancy buffers by size
  std::vector<uint32_t *> occ_retired;         // of requests that did not finish (freed at destroy)

  Batch batches[2];
  int next_batch = 0;

  // out of core: the shared brick pool and the worker that renders requests
  // on host-brick volumes
  char *brick_pool = nullptr;
  BrickArena *arena = nullptr;
  std::thread ooc_thread;
  std::condition_variable cv_ooc;
  std::deque<uint64_t> ooc_queue;    // admitted out-of-core tickets
  hipStream_t ooc_stream = nullptr;
  float *ooc_tf = nullptr;           // device TF staging of the worker
  float *ooc_tf_host = nullptr;      // pinned

  // stats
  uint64_t n_submitted = 0, n_admitted = 0, n_completed = 0, n_rejected = 0, n_launches = 0, n_items = 0;
  std::vector<double> latencies_ms;
  double busy_s = 0, busy_since = -1;
  uint64_t pixels_done = 0, samples_done = 0;
  // queue length over time (since the last reset)
  double q_area = 0, q_since = 0, q_last = 0;
  uint64_t q_max = 0;
};

namespace {

void charge(vr_server *s, size_t bytes) {
  s->hbm_used += bytes;
  s->hbm_peak = std::max(s->hbm_peak, s->hbm_used);
}

// Account the queue length up to now (call before the queue changes and
// after, lock held).
void note_queue(vr_server *s) {
  const double t = now_s();
  s->q_area += (double)s->queue.size() * (t - s->q_last);
  s->q_last = t;
  s->q_max = std::max<uint64_t>(s->q_max, s->queue.size());
}

// Free pooled buffers (largest first) until `bytes` more fit the budget.
// Lock held.  Returns whether they fit.
bool make_room(vr_server *s, size_t bytes) {
  while (s->hbm_used + bytes > s->cfg.hbm_budget_bytes && (!s->image_pool.empty() || !s->occ_pool.empty())) {
    const bool img = !s->image_pool.empty() &&
                     (s->occ_pool.empty() || std::prev(s->image_pool.end())->first >= std::prev(s->occ_pool.end())->first);
    if (img) {
      auto big = std::prev(s->image_pool.end());
      (void)s->ops->dev_free(big->second);
      s->hbm_used -= big->first;
      s->image_pool.erase(big);
    } else {
      auto big = std::prev(s->occ_pool.end());
      (void)s->ops->dev_free(big->second);
      s->hbm_used -= big->first;
      s->occ_pool.erase(big);
    }
  }
  return s->hbm_used + bytes <= s->cfg.hbm_budget_bytes;
}

// Device bytes a request holds while admitted: its result image and, when it
// skips, the occupancy buffer of its volume's block grid.
size_t request_bytes(const vr_server *s, int32_t volume_id, size_t image_bytes, bool skip) {
  auto it = s->volumes.find(volume_id);
  size_t b = image_bytes;
  if (skip && it != s->volumes.end() && !it->second.bricked && it->second.vc.minmax)
    b += occupancy_bytes(it->second.vc);
  return b;
}

// Get a buffer of exactly `bytes` from `pool`, else a new allocation if the
// budget allows (evicting pooled buffers of other sizes).  Lock held.
// Returns nullptr when the budget is full.
template <class T>
T *acquire(vr_server *s, std::multimap<size_t, T *> &pool, size_t bytes) {
  auto it = pool.find(bytes);
  if (it != pool.end()) {
    T *p = it->second;
    pool.erase(it);
    return p;
  }
  if (!make_room(s, bytes)) return nullptr;
  T *p = nullptr;
  if (s->ops->dev_alloc(reinterpret_cast<void **>(&p), bytes) != hipSuccess) return nullptr;
  charge(s, bytes);
  return p;
}

void release_image(vr_server *s, float *p, size_t bytes) {
  if (p) s->image_pool.emplace(bytes, p);
}

size_t batch_capacity(const vr_serve_config &c) {
  return (size_t)c.max_inflight * (align16(sizeof(ServeSlot)) + (size_t)VR_MAX_TF_NODES * 16) +
         (size_t)c.max_batch_tiles * sizeof(ServeItem) + 64 + 16;
}

void fail_all(vr_server *s, vr_status st) {
  s->dead = true;
  s->dead_status = st;
  for (auto &kv : s->requests) {
    Request &r = *kv.second;
    if (r.state == RState::Queued || r.state == RState::Admitted) {
      r.state = RState::Failed;
      r.error = st;
      s->volumes[r.volume_id].users--;
    }
  }
  note_queue(s);
  s->queue.clear();
  note_queue(s);
  s->admitted.clear();
  s->cv_done.notify_all();
}

// FIFO admission; lock held.  A head request that can never fit next to the
// resident volumes (volumes were added after it was queued) fails with
// VR_E_BUDGET instead of blocking the queue.
void admit(vr_server *s) {
  while (!s->queue.empty() && (int32_t)s->admitted.size() < s->cfg.max_inflight) {
    Request &r = *s->requests[s->queue.front()];
    const bool skip = !r.out_of_core && r.mc.skip && s->volumes[r.volume_id].vc.minmax;
    const size_t need = request_bytes(s, r.volume_id, r.image_bytes, r.mc.skip != 0);
    if (s->resident_bytes + need > s->cfg.hbm_budget_bytes) {
      note_queue(s);
      s->queue.pop_front();
      note_queue(s);
      r.state = RState::Failed;
      r.error = VR_E_BUDGET;
      s->volumes[r.volume_id].users--;
      s->n_rejected++;
      s->cv_done.notify_all();
      continue;
    }
    float *img = acquire(s, s->image_pool, r.image_bytes);
    if (!img) break;  // head of line waits for memory
    uint32_t *occ = nullptr;
    if (skip) {
      const size_t ob = occupancy_bytes(s->volumes[r.volume_id].vc);
      occ = acquire(s, s->occ_pool, ob);
      if (!occ) {
        release_image(s, img, r.image_bytes);
        break;  // waits for memory
      }
      r.occ = occ;
      r.occ_bytes = ob;
      r.occ_radius = s->volumes[r.volume_id].radius_fits ? kEmptyRadiusMax : 0;
      r.occ_batch = -1;  // computed by the first batch that carries the request
    }
    r.image = img;
    r.state = RState::Admitted;
    note_queue(s);
    s->queue.pop_front();
    note_queue(s);
    s->admitted.push_back(r.ticket);
    s->n_admitted++;
    if (r.out_of_core) {
      s->ooc_queue.push_back(r.ticket);
      s->cv_ooc.notify_one();
    }
  }
}

// Finish a request the worker rendered; lock held.
void complete(vr_server *s, Request &r, vr_status st) {
  const double t = now_s();
  if (r.state != RState::Admitted) {  // failed or cancelled meanwhile (its slot is already freed)
    s->cv_done.notify_all();
    return;
  }
  auto at = std::find(s->admitted.begin(), s->admitted.end(), r.ticket);
  if (at != s->admitted.end()) s->admitted.erase(at);
  s->volumes[r.volume_id].users--;
  if (st == VR_OK) {
    r.state = RState::Done;
    r.t_done = t;
    s->latencies_ms.push_back((r.t_done - r.t_submit) * 1e3);
    s->n_completed++;
    s->pixels_done += (uint64_t)r.cam.W * r.cam.H;
  } else {
    r.state = RState::Failed;
    r.error = st;
  }
  s->cv_done.notify_all();
  s->cv_work.notify_one();  // a slot is free
}

// The out-of-core worker: renders admitted requests on host-brick volumes
// one at a time (they share the brick pool), through vr_bricked_render on
// its own stream.
void ooc_worker(vr_server *s) {
  (void)s->ops->set_device(s->cfg.device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    s->cv_ooc.wait(lk, [&] { return s->stop || !s->ooc_queue.empty(); });
    if (s->ooc_queue.empty()) break;  // stop requested and nothing left
    const uint64_t t = s->ooc_queue.front();
    s->ooc_queue.pop_front();
    auto it = s->requests.find(t);
    if (it == s->requests.end()) continue;
    Request &r = *it->second;
    if (r.state != RState::Admitted) continue;  // cancelled meanwhile
    if (s->stop) {
      r.state = RState::Cancelled;
      s->admitted.erase(std::find(s->admitted.begin(), s->admitted.end(), r.ticket));
      s->volumes[r.volume_id].users--;
      s->cv_done.notify_all();
      continue;
    }
    vr_bricked *bv = s->volumes[r.volume_id].bricked;
    const size_t tf_bytes = (size_t)r.K * 16;
    memcpy(s->ooc_tf_host, r.tf.data(), tf_bytes);
    const vr_camera cam = r.cam_desc;
    vr_params p{};
    p.step = r.mc.step;
    p.ert_threshold = r.mc.ert;
    p.use_skip = 1;
    p.filter = VR_FILTER_BSPLINE;
    p.counters = nullptr;
    vr_tf tf{s->ooc_tf, r.K, r.v0, r.v1};
    float *image = r.image;
    lk.unlock();  // the volume stays registered: this request counts as its user
    vr_status st = VR_OK;
    hipError_t e = s->ops->copy_async(s->ooc_tf, s->ooc_tf_host, tf_bytes, hipMemcpyHostToDevice, s->ooc_stream);
    if (e != hipSuccess) st = hip_fail(e, "out-of-core TF upload");
    if (st == VR_OK) st = vr_bricked_render(bv, &cam, 1, &tf, &p, image, s->ooc_stream);
    if (st == VR_OK && (e = s->ops->stream_sync(s->ooc_stream)) != hipSuccess)
      st = hip_fail(e, "out-of-core render");
    lk.lock();
    complete(s, r, st);
  }
}

// Retire a finished batch; lock held.
void retire(vr_server *s, Batch &b) {
  double t = now_s();
  s->samples_done += *b.samples_host;
  for (auto &pr : b.per_request) {
    auto it = s->requests.find(pr.first);
    if (it == s->requests.end()) continue;
    Request &r = *it->second;
    r.items_done += pr.second;
    if (r.state == RState::Admitted && r.items_done == r.items_total) {
      r.state = RState::Done;
      r.t_done = t;
      s->latencies_ms.push_back((r.t_done - r.t_submit) * 1e3);
      s->n_completed++;
      s->pixels_done += (uint64_t)r.cam.W * r.cam.H;
      s->admitted.erase(std::find(s->admitted.begin(), s->admitted.end(), r.ticket));
      s->volumes[r.volume_id].users--;
      if (r.occ) {  // every batch that read it has finished
        s->occ_pool.emplace(r.occ_bytes, r.occ);
        r.occ = nullptr;
      }
    }
  }
  b.per_request.clear();
  b.busy = false;
  s->cv_done.notify_all();
}

// Fill and launch batch `b` from the admitted requests; lock held.
// Returns false if there was nothing to issue.
bool issue(vr_server *s, Batch &b) {
  std::vector<uint64_t> live;
  for (uint64_t t : s->admitted) {
    Request &r = *s->requests[t];
    if (!r.out_of_core && r.items_issued < r.items_total) live.push_back(t);
  }
  if (live.empty()) return false;
  const int32_t cap_items = s->cfg.max_batch_tiles;
  // items per request: round-robin shares of the launch
  std::vector<int64_t> take(live.size(), 0);
  int64_t left = cap_items;
  bool progress = true;
  const size_t n = live.size();
  while (left > 0 && progress) {
    progress = false;
    int64_t share = std::max<int64_t>(1, left / (int64_t)n);
    for (size_t q = 0; q < n && left > 0; ++q) {
      size_t i = (s->rr + q) % n;
      Request &r = *s->requests[live[i]];
      int64_t rem = r.items_total - r.items_issued - take[i];
      int64_t t = std::min<int64_t>({rem, share, left});
      if (t > 0) {
        take[i] += t;
        left -= t;
        progress = true;
      }
    }
  }
  s->rr = (s->rr + 1) % std::max<size_t>(1, n);
  // lay out slots, TF tables and items in the pinned staging buffer
  std::vector<size_t> slot_of;
  size_t n_slots = 0;
  for (size_t i = 0; i < n; ++i)
    if (take[i] > 0) ++n_slots;
  size_t off_slots = 0;
  size_t off_tf = align16(n_slots * sizeof(ServeSlot));
  size_t tf_bytes = 0;
  for (size_t i = 0; i < n; ++i)
    if (take[i] > 0) tf_bytes += align16((size_t)s->requests[live[i]]->K * 16);
  size_t off_items = off_tf + tf_bytes;
  int64_t n_items_total = cap_items - left;
  size_t off_count = align16(off_items + (size_t)n_items_total * sizeof(ServeItem));
  size_t total = off_count + sizeof(unsigned long long);
  if (total > b.cap) return false;  // cannot happen: capacity covers the worst case
  ServeSlot *slots = reinterpret_cast<ServeSlot *>(b.host + off_slots);
  ServeItem *items = reinterpret_cast<ServeItem *>(b.host + off_items);
  size_t tf_cursor = off_tf;
  int32_t slot = 0;
  int64_t item = 0;
  int32_t max_k = 2;
  b.per_request.clear();
  b.pixels = 0;
  const int bi = (int)(&b - s->batches);
  Batch &other = s->batches[bi ^ 1];
  b.gen++;
  std::vector<std::pair<Request *, size_t>> occ_new;  // requests whose occupancy this batch computes, TF offset
  bool wait_other = false;
  std::vector<std::pair<float, ServeItem>> keyed;
  keyed.reserve((size_t)n_items_total);
  for (size_t i = 0; i < n; ++i) {
    if (take[i] == 0) continue;
    Request &r = *s->requests[live[i]];
    Volume &v = s->volumes[r.volume_id];
    ServeSlot &sl = slots[slot];
    sl.vol = v.vc;
    sl.cam = r.cam;
    sl.mc = r.mc;
    sl.out = r.image;
    sl.tf.K = r.K;
    max_k = std::max(max_k, r.K);
    sl.tf.v0 = r.v0;
    sl.tf.scale = (float)(r.K - 1) / (r.v1 - r.v0);
    sl.tf.status = nullptr;  // validated at submit
    memcpy(b.host + tf_cursor, r.tf.data(), (size_t)r.K * 16);
    sl.tf.table = reinterpret_cast<const float *>(b.dev + tf_cursor);
    if (r.occ && r.occ_batch < 0) {
      r.occ_batch = bi;
      r.occ_gen = b.gen;
      occ_new.emplace_back(&r, tf_cursor);
    } else if (r.occ && r.occ_batch == (bi ^ 1) && other.busy && other.gen == r.occ_gen) {
      wait_other = true;  // computed by the other batch, which may still run
    }
    sl.vol.occ = r.occ;
    sl.vol.occ_radius = r.occ ? r.occ_radius : 0;
    tf_cursor += align16((size_t)r.K * 16);
    for (int64_t q = 0; q < take[i]; ++q) {
      const int64_t rank = r.items_issued + q;
      const int32_t id = r.order[(size_t)rank];
      ServeItem it;
      it.slot = slot;
      it.sx = (int16_t)(id % r.stx);
      it.sy = (int16_t)(id / r.stx);
      // heavy (central) tiles of every request first: merge by relative rank
      keyed.emplace_back((float)rank / (float)r.items_total, it);
      ++item;
    }
    r.items_issued += take[i];
    b.per_request.emplace_back(r.ticket, (int32_t)take[i]);
    b.pixels += take[i] * kSuperEdge * kSuperEdge;
    ++slot;
  }
  std::stable_sort(keyed.begin(), keyed.end(),
                   [](const std::pair<float, ServeItem> &a, const std::pair<float, ServeItem> &c) { return a.first < c.first; });
  for (size_t q = 0; q < keyed.size(); ++q) items[q] = keyed[q].second;
  *reinterpret_cast<unsigned long long *>(b.host + off_count) = 0;  // the launch's sample counter
  hipError_t e = s->ops->copy_async(b.dev, b.host, total, hipMemcpyHostToDevice, b.stream);
  for (auto &rn : occ_new) {  // from the TF tables just copied
    if (e != hipSuccess) break;
    Request &r = *rn.first;
    const Volume &v = s->volumes[r.volume_id];
    TfConst tc;
    tc.table = reinterpret_cast<const float *>(b.dev + rn.second);
    tc.K = r.K;
    tc.v0 = r.v0;
    tc.scale = (float)(r.K - 1) / (r.v1 - r.v0);
    tc.status = nullptr;
    e = s->ops->occupancy(v.vc, tc, r.occ, r.occ_radius > 0, b.stream);
  }
  if (e == hipSuccess) e = s->ops->event_record(b.occ_done, b.stream);
  if (e == hipSuccess && wait_other) e = s->ops->stream_wait(b.stream, other.occ_done);
  if (e == hipSuccess)
    e = s->ops->launch_batch(reinterpret_cast<const ServeSlot *>(b.dev + off_slots),
                           reinterpret_cast<const ServeItem *>(b.dev + off_items), (int32_t)item, max_k,
                           reinterpret_cast<unsigned long long *>(b.dev + off_count), b.stream);
  if (e == hipSuccess)
    e = s->ops->copy_async(b.samples_host, b.dev + off_count, sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           b.stream);
  if (e == hipSuccess) e = s->ops->event_record(b.done, b.stream);
  if (e != hipSuccess) {
    fail(VR_E_DEVICE, "serve launch: %s", hipGetErrorString(e));
    fail_all(s, VR_E_DEVICE);
    return false;
  }
  b.busy = true;
  s->n_launches++;
  s->n_items += (uint64_t)item;
  return true;
}

void scheduler(vr_server *s) {
  (void)s->ops->set_device(s->cfg.device);
  std::unique_lock<std::mutex> lk(s->mu);
  while (!s->stop) {
    admit(s);
    for (int q = 0; q < 2 && !s->dead; ++q) {
      Batch &b = s->batches[s->next_batch];
      if (b.busy || !issue(s, b)) break;
      s->next_batch ^= 1;
    }
    bool retired = false;
    for (Batch &b : s->batches) {
      if (!b.busy) continue;
      hipError_t e = s->ops->event_query(b.done);
      if (e == hipSuccess) {
        retire(s, b);
        retired = true;
      } else if (e != hipErrorNotReady) {
        fail(VR_E_DEVICE, "serve batch: %s", hipGetErrorString(e));
        b.busy = false;
        fail_all(s, VR_E_DEVICE);
      }
    }
    const bool any_busy = s->batches[0].busy || s->batches[1].busy;
    const double t = now_s();
    if (any_busy && s->busy_since < 0) s->busy_since = t;
    if (!any_busy && s->busy_since >= 0) {
      s->busy_s += t - s->busy_since;
      s->busy_since = -1;
    }
    if (retired) continue;
    if (any_busy)
      s->cv_work.wait_for(lk, std::chrono::microseconds(20));
    else
      s->cv_work.wait(lk);
  }
}

// Device memory, streams, events and pinned buffers the server holds (also
// after a failed create); lock not needed (no thread runs).
void free_server_resources(vr_server *s) {
  const ServeOps *o = s->ops;
  for (Batch &b : s->batches) {
    if (b.done) (void)o->event_destroy(b.done);
    if (b.occ_done) (void)o->event_destroy(b.occ_done);
    if (b.stream) (void)o->stream_destroy(b.stream);
    if (b.host) (void)o->host_free(b.host);
    if (b.samples_host) (void)o->host_free(b.samples_host);
    if (b.dev) (void)o->dev_free(b.dev);
  }
  for (auto &kv : s->requests) {
    if (kv.second->image) (void)o->dev_free(kv.second->image);
    if (kv.second->occ) (void)o->dev_free(kv.second->occ);
  }
  for (auto &kv : s->image_pool) (void)o->dev_free(kv.second);
  for (auto &kv : s->occ_pool) (void)o->dev_free(kv.second);
  for (uint32_t *p : s->occ_retired) (void)o->dev_free(p);
  for (auto &kv : s->volumes) {
    if (kv.second.blocks) o->free_blocks(kv.second.blocks);
    if (kv.second.bricked) vr_bricked_free(kv.second.bricked);
  }
  if (s->ooc_stream) (void)o->stream_destroy(s->ooc_stream);
  if (s->ooc_tf) (void)o->dev_free(s->ooc_tf);
  if (s->ooc_tf_host) (void)o->host_free(s->ooc_tf_host);
  if (s->brick_pool) (void)o->dev_free(s->brick_pool);
  brick_arena_delete(s->arena);
}

hipError_t hip_device_count(int *n) { return hipGetDeviceCount(n); }
hipError_t hip_set_device(int d) { return hipSetDevice(d); }
hipError_t hip_stream_create(hipStream_t *st) { return hipStreamCreateWithFlags(st, hipStreamNonBlocking); }
hipError_t hip_stream_destroy(hipStream_t st) { return hipStreamDestroy(st); }
hipError_t hip_stream_sync(hipStream_t st) { return hipStreamSynchronize(st); }
hipError_t hip_event_create(hipEvent_t *e) { return hipEventCreateWithFlags(e, hipEventDisableTiming); }
hipError_t hip_event_destroy(hipEvent_t e) { return hipEventDestroy(e); }
hipError_t hip_event_record(hipEvent_t e, hipStream_t st) { return hipEventRecord(e, st); }
hipError_t hip_event_query(hipEvent_t e) { return hipEventQuery(e); }
hipError_t hip_stream_wait(hipStream_t st, hipEvent_t e) { return hipStreamWaitEvent(st, e, 0); }
hipError_t hip_dev_alloc(void **p, size_t n) {
  const hipError_t e = hipMalloc(p, n);
  if (e != hipSuccess) (void)hipGetLastError();
  return e;
}
hipError_t hip_dev_free(void *p) { return hipFree(p); }
hipError_t hip_host_alloc(void **p, size_t n) { return hipHostMalloc(p, n, hipHostMallocDefault); }
hipError_t hip_host_free(void *p) { return hipHostFree(p); }
hipError_t hip_copy_async(void *dst, const void *src, size_t n, hipMemcpyKind k, hipStream_t st) {
  return hipMemcpyAsync(dst, src, n, k, st);
}
hipError_t hip_occupancy(const VolConst &v, const TfConst &tf, uint32_t *bits, bool radius, hipStream_t st) {
  return radius ? launch_occupancy_planes(v, tf, bits, st) : launch_occupancy_bits(v, tf, bits, st);
}
vr_status hip_build_blocks(const vr_volume *vol, int32_t edge, vr_blocks **out, VolConst *vc) {
  vr_blocks *blocks = nullptr;
  vr_status st = check_volume(vol, vc);
  if (st) return st;
  if ((st = vr_build_blocks(vol, edge, nullptr, &blocks))) return st;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    vr_blocks_free(blocks);
    return hip_fail(e, "block build");
  }
  if ((st = attach_blocks(blocks, vol, vc))) {
    vr_blocks_free(blocks);
    return st;
  }
  *out = blocks;
  return VR_OK;
}

const ServeOps kHipOps = {hip_device_count, hip_set_device,  hip_stream_create, hip_stream_destroy, hip_stream_sync,
                          hip_event_create, hip_event_destroy, hip_event_record, hip_event_query,    hip_stream_wait,
                          hip_dev_alloc,    hip_dev_free,    hip_host_alloc,    hip_host_free,      hip_copy_async,
                          hip_occupancy,    launch_serve_batch, hip_build_blocks, vr_blocks_free};

}  // namespace

namespace vr {

const ServeOps *serve_hip_ops() { return &kHipOps; }

vr_status serve_create_with_ops(const vr_serve_config *cfg, const ServeOps *ops, vr_server **out) {
  if (!cfg || !out || !ops) return fail(VR_E_INVALID_ARG, "config or out is NULL");
  *out = nullptr;
  if (cfg->max_inflight < 1 || cfg->max_inflight > 1024) return fail(VR_E_INVALID_ARG, "max_inflight outside [1, 1024]");
  if (cfg->max_batch_tiles < 0 || cfg->max_batch_tiles > (1 << 20)) return fail(VR_E_INVALID_ARG, "max_batch_tiles outside [0, 2^20]");
  if (cfg->hbm_budget_bytes == 0) return fail(VR_E_INVALID_ARG, "hbm_budget_bytes is zero");
  int ndev = 0;
  if (ops->device_count(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev)
    return fail(VR_E_INVALID_ARG, "device %d not available", cfg->device);
  std::unique_ptr<vr_server> s(new (std::nothrow) vr_server());
  if (!s) return fail(VR_E_OOM, "host allocation failed");
  s->cfg = *cfg;
  s->ops = ops;
  if (s->cfg.max_batch_tiles == 0) s->cfg.max_batch_tiles = 2048;
  hipError_t e = ops->set_device(cfg->device);
  vr_status st = VR_OK;
  if (e != hipSuccess) st = hip_fail(e, "set device");
  const size_t cap = batch_capacity(s->cfg);
  for (Batch &b : s->batches) {
    if (st) break;
    b.cap = cap;
    if ((e = ops->stream_create(&b.stream)) != hipSuccess || (e = ops->event_create(&b.done)) != hipSuccess ||
        (e = ops->event_create(&b.occ_done)) != hipSuccess)
      st = hip_fail(e, "stream or event");
    else if ((e = ops->host_alloc((void **)&b.host, cap)) != hipSuccess ||
             (e = ops->host_alloc((void **)&b.samples_host, sizeof(unsigned long long))) != hipSuccess)
      st = hip_fail(e, "pinned staging");
    else if ((e = ops->dev_alloc((void **)&b.dev, cap)) != hipSuccess)
      st = fail(VR_E_OOM, "device staging: %s", hipGetErrorString(e));
    else
      *b.samples_host = 0;
  }
  if (!st && (e = ops->stream_create(&s->ooc_stream)) != hipSuccess) st = hip_fail(e, "stream");
  if (!st && (e = ops->dev_alloc((void **)&s->ooc_tf, (size_t)VR_MAX_TF_NODES * 16)) != hipSuccess)
    st = fail(VR_E_OOM, "TF staging: %s", hipGetErrorString(e));
  if (!st && (e = ops->host_alloc((void **)&s->ooc_tf_host, (size_t)VR_MAX_TF_NODES * 16)) != hipSuccess)
    st = hip_fail(e, "pinned TF staging");
  if (st) {
    free_server_resources(s.get());
    return st;
  }
  s->q_since = s->q_last = now_s();
  vr_server *raw = s.release();
  raw->thread = std::thread(scheduler, raw);
  raw->ooc_thread = std::thread(ooc_worker, raw);
  *out = raw;
  return VR_OK;
}

}  // namespace vr

extern "C" {

vr_status vr_serve_create(const vr_serve_config *cfg, vr_server **out) {
  return serve_create_with_ops(cfg, serve_hip_ops(), out);
}

vr_status vr_serve_add_volume(vr_server *s, const vr_volume *vol, int32_t block_edge, int32_t *volume_id) {
  if (!s || !volume_id) return fail(VR_E_INVALID_ARG, "server or volume_id is NULL");
  VolConst vc;
  vr_status st = check_volume(vol, &vc);
  if (st) return st;
  vr_blocks *blocks = nullptr;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(VR_E_SHUTDOWN, "server is shutting down");
  }
  (void)s->ops->set_device(s->cfg.device);
  if ((st = s->ops->build_blocks(vol, block_edge, &blocks, &vc))) return st;
  std::lock_guard<std::mutex> lk(s->mu);
  // the volume's own memory (caller-owned, resident) and its blocks (plain and widened ranges)
  const size_t vb = (size_t)vc.bytes;
  const size_t bb = 2 * (size_t)vc.nbx * vc.nby * vc.nbz * sizeof(float2);
  if (!make_room(s, vb + bb)) {
    s->ops->free_blocks(blocks);
    return fail(VR_E_BUDGET, "volume (%zu bytes) and blocks (%zu bytes) do not fit the HBM budget (%llu of %llu bytes held)",
                vb, bb, (unsigned long long)s->hbm_used, (unsigned long long)s->cfg.hbm_budget_bytes);
  }
  charge(s, vb + bb);
  s->resident_bytes += vb + bb;
  int32_t id = s->next_volume++;
  Volume &v = s->volumes[id];
  v.desc = *vol;
  v.vc = vc;
  v.radius_fits = occupancy_planes_fit(vc, VR_MAX_TF_NODES);
  v.blocks = blocks;
  v.resident_bytes = vb + bb;
  *volume_id = id;
  return VR_OK;
}

vr_status vr_serve_add_host_volume(vr_server *s, const vr_volume *host_vol, int32_t brick_edge, int32_t *volume_id) {
  if (!s || !volume_id) return fail(VR_E_INVALID_ARG, "server or volume_id is NULL");
  if (s->cfg.brick_pool_bytes == 0) return fail(VR_E_INVALID_ARG, "the server was created without a brick pool");
  (void)s->ops->set_device(s->cfg.device);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) return fail(VR_E_SHUTDOWN, "server is shutting down");
    if (!s->arena) {
      if (!make_room(s, s->cfg.brick_pool_bytes))
        return fail(VR_E_BUDGET, "the brick pool (%llu bytes) does not fit the HBM budget",
                    (unsigned long long)s->cfg.brick_pool_bytes);
      char *mem = nullptr;
      hipError_t e = s->ops->dev_alloc((void **)&mem, (size_t)s->cfg.brick_pool_bytes);
      if (e != hipSuccess) return fail(VR_E_OOM, "brick pool: %s", hipGetErrorString(e));
      BrickArena *a = brick_arena_new(mem, s->cfg.brick_pool_bytes);
      if (!a) {
        (void)s->ops->dev_free(mem);
        return fail(VR_E_OOM, "host allocation failed");
      }
      s->brick_pool = mem;
      s->arena = a;
      charge(s, s->cfg.brick_pool_bytes);
      s->resident_bytes += s->cfg.brick_pool_bytes;
    }
  }
  // pinned host bricks and their device structures (the pool is the arena's;
  // the worker's renders take turns in it)
  vr_bricked *bv = nullptr;
  vr_status st = bricked_create(host_vol, brick_edge, 0, s->arena, &bv);
  if (st) return st;
  std::lock_guard<std::mutex> lk(s->mu);
  const size_t db = (size_t)bricked_device_bytes(bv);
  if (!make_room(s, db)) {
    vr_bricked_free(bv);
    return fail(VR_E_BUDGET, "the out-of-core volume's block structures (%zu bytes) do not fit the HBM budget", db);
  }
  charge(s, db);
  s->resident_bytes += db;
  int32_t id = s->next_volume++;
  Volume &v = s->volumes[id];
  v.desc = *host_vol;
  v.desc.data = nullptr;  // host memory, read at registration only
  memset(&v.vc, 0, sizeof(v.vc));
  v.vc.nx = (int32_t)host_vol->nx;
  v.vc.ny = (int32_t)host_vol->ny;
  v.vc.nz = (int32_t)host_vol->nz;
  v.bricked = bv;
  v.resident_bytes = db;
  *volume_id = id;
  return VR_OK;
}

vr_status vr_serve_remove_volume(vr_server *s, int32_t volume_id) {
  if (!s) return fail(VR_E_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->volumes.find(volume_id);
  if (it == s->volumes.end()) return fail(VR_E_NOT_FOUND, "unknown volume %d", volume_id);
  if (it->second.users > 0) return fail(VR_E_BUSY, "volume %d has %lld requests queued or in flight", volume_id, (long long)it->second.users);
  if (it->second.bricked) vr_bricked_free(it->second.bricked);
  if (it->second.blocks) s->ops->free_blocks(it->second.blocks);
  s->hbm_used -= it->second.resident_bytes;
  s->resident_bytes -= it->second.resident_bytes;
  s->volumes.erase(it);
  return VR_OK;
}

vr_status vr_serve_submit(vr_server *s, const vr_request *req, uint64_t *ticket) {
  if (!s || !req || !ticket) return fail(VR_E_INVALID_ARG, "server, request or ticket is NULL");
  std::unique_ptr<Request> r(new Request());
  vr_status st = check_camera(&req->cam, &r->cam);
  if (st) return st;
  r->cam_desc = req->cam;
  if (!req->tf_table_host) return fail(VR_E_INVALID_ARG, "tf_table_host is NULL");
  if (req->K < 2 || req->K > VR_MAX_TF_NODES) return fail(VR_E_INVALID_ARG, "TF node count K=%d outside [2, %d]", req->K, VR_MAX_TF_NODES);
  if (!std::isfinite(req->tf_v0) || !std::isfinite(req->tf_v1) || !(req->tf_v1 > req->tf_v0))
    return fail(VR_E_INVALID_ARG, "TF value range must be finite with v1 > v0");
  r->tf.assign(req->tf_table_host, req->tf_table_host + (size_t)req->K * 4);
  for (int32_t j = 0; j < req->K; ++j) {
    for (int c = 0; c < 4; ++c)
      if (!std::isfinite(r->tf[4 * j + c])) return fail(VR_E_INVALID_ARG, "TF entry %d is not finite", j);
    if (r->tf[4 * j + 3] < 0.0f) return fail(VR_E_INVALID_ARG, "TF node %d has negative extinction", j);
  }
  if ((st = check_march(req->step, req->ert_threshold, req->use_skip, &r->mc))) return st;
  r->K = req->K;
  r->v0 = req->tf_v0;
  r->v1 = req->tf_v1;
  r->volume_id = req->volume_id;
  r->image_bytes = (size_t)req->cam.width * req->cam.height * 16;
  r->stx = (req->cam.width + kSuperEdge - 1) / kSuperEdge;
  r->sty = (req->cam.height + kSuperEdge - 1) / kSuperEdge;
  if (r->stx > 32767 || r->sty > 32767) return fail(VR_E_UNSUPPORTED, "image too large for serving");
  r->items_total = (int64_t)r->stx * r->sty;
  // centre-out tile order (the volume's projected centre; image centre if it does not project)
  double centre[3] = {0.0, 0.0, 0.0};
  {
    std::lock_guard<std::mutex> lk0(s->mu);
    auto vit0 = s->volumes.find(req->volume_id);
    if (vit0 != s->volumes.end()) {
      centre[0] = 0.5 * (double)(vit0->second.desc.nx - 1);
      centre[1] = 0.5 * (double)(vit0->second.desc.ny - 1);
      centre[2] = 0.5 * (double)(vit0->second.desc.nz - 1);
    }
  }
  {
    const CamConst &c = r->cam;
    double d[3], x = 0.0, y = 0.0, z = 0.0;
    for (int k = 0; k < 3; ++k) d[k] = centre[k] - c.eye[k];
    for (int k = 0; k < 3; ++k) {
      z += d[k] * c.fwd[k];
      x += d[k] * c.right[k];
      y += d[k] * c.up[k];
    }
    double sx = 0.0, sy = 0.0;
    if (c.proj != 0) {
      if (z > 0.0) {
        sx = x / (z * c.th * ((double)c.W / (double)c.H));
        sy = y / (z * c.th);
      }
    } else {
      sx = c.hw > 0.0 ? x / c.hw : 0.0;
      sy = c.hh > 0.0 ? y / c.hh : 0.0;
    }
    const double cx = std::fmin(std::fmax(((sx + 1.0) * 0.5 * c.W) / kSuperEdge - 0.5, -1e6), 1e6);
    const double cy = std::fmin(std::fmax(((1.0 - sy) * 0.5 * c.H) / kSuperEdge - 0.5, -1e6), 1e6);
    std::vector<std::pair<float, int32_t>> kd((size_t)r->items_total);
    for (int32_t t = 0; t < (int32_t)r->items_total; ++t)
      kd[(size_t)t] = {(float)std::hypot((double)(t % r->stx) - cx, (double)(t / r->stx) - cy), t};
    std::sort(kd.begin(), kd.end());
    r->order.resize(kd.size());
    for (size_t q = 0; q < kd.size(); ++q) r->order[q] = kd[q].second;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return fail(VR_E_SHUTDOWN, "server is shutting down");
  if (s->dead) return fail(s->dead_status, "server failed earlier");
  auto vit = s->volumes.find(req->volume_id);
  if (vit == s->volumes.end()) {
    s->n_rejected++;
    return fail(VR_E_NOT_FOUND, "unknown volume %d", req->volume_id);
  }
  const size_t need = request_bytes(s, req->volume_id, r->image_bytes, r->mc.skip != 0);
  if (s->resident_bytes + need > s->cfg.hbm_budget_bytes) {
    s->n_rejected++;
    return fail(VR_E_BUDGET,
                "the request needs %zu device bytes (image and occupancy buffer); %llu of the %llu-byte budget are "
                "held by resident volumes and blocks",
                need, (unsigned long long)s->resident_bytes, (unsigned long long)s->cfg.hbm_budget_bytes);
  }
  Volume &v = vit->second;
  r->out_of_core = v.bricked != nullptr;
  if (r->out_of_core) r->items_total = 0;  // rendered by the out-of-core worker
  r->ticket = s->next_ticket++;
  r->t_submit = now_s();
  v.users++;
  *ticket = r->ticket;
  note_queue(s);
  s->queue.push_back(r->ticket);
  note_queue(s);
  s->requests.emplace(r->ticket, std::move(r));
  s->n_submitted++;
  s->cv_work.notify_one();
  return VR_OK;
}

vr_status vr_serve_wait(vr_server *s, uint64_t ticket, int64_t timeout_us, const float **rgba_device) {
  if (!s) return fail(VR_E_INVALID_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->requests.find(ticket);
  if (it == s->requests.end()) return fail(VR_E_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
  Request *r = it->second.get();
  auto ready = [&] { return r->state == RState::Done || r->state == RState::Cancelled || r->state == RState::Failed; };
  s->waiters++;
  bool ok = true;
  if (timeout_us < 0)
    s->cv_done.wait(lk, ready);
  else
    ok = s->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
  s->waiters--;
  if (s->waiters == 0) s->cv_done.notify_all();
  if (!ok)
    return fail(VR_E_TIMEOUT, "ticket %llu not complete after %lld us", (unsigned long long)ticket, (long long)timeout_us);
  if (r->state == RState::Cancelled) return fail(VR_E_SHUTDOWN, "ticket %llu cancelled by shutdown", (unsigned long long)ticket);
  if (r->state == RState::Failed) return fail(r->error, "ticket %llu failed", (unsigned long long)ticket);
  if (rgba_device) *rgba_device = r->image;
  return VR_OK;
}

vr_status vr_serve_release(vr_server *s, uint64_t ticket) {
  if (!s) return fail(VR_E_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->requests.find(ticket);
  if (it == s->requests.end()) return fail(VR_E_NOT_FOUND, "unknown ticket %llu", (unsigned long long)ticket);
  Request &r = *it->second;
  if (r.state == RState::Queued || r.state == RState::Admitted)
    return fail(VR_E_BUSY, "ticket %llu is not complete", (unsigned long long)ticket);
  release_image(s, r.image, r.image_bytes);
  if (r.occ) s->occ_retired.push_back(r.occ);  // a cancelled request's batches may still read it
  s->requests.erase(it);
  s->cv_work.notify_one();
  return VR_OK;
}

vr_status vr_serve_stats_get(vr_server *s, vr_serve_stats *o) {
  if (!s || !o) return fail(VR_E_INVALID_ARG, "server or out is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  memset(o, 0, sizeof(*o));
  o->submitted = s->n_submitted;
  o->admitted = s->n_admitted;
  o->completed = s->n_completed;
  o->rejected = s->n_rejected;
  o->queued = s->queue.size();
  o->inflight = s->admitted.size();
  o->hbm_used = s->hbm_used;
  o->hbm_peak = s->hbm_peak;
  o->launches = s->n_launches;
  o->tiles = s->n_items;
  std::vector<double> l = s->latencies_ms;
  if (!l.empty()) {
    std::sort(l.begin(), l.end());
    auto pct = [&](double p) {
      double idx = p * (double)(l.size() - 1);
      size_t lo = (size_t)std::floor(idx), hi = (size_t)std::ceil(idx);
      return l[lo] + (l[hi] - l[lo]) * (idx - (double)lo);
    };
    o->p50_ms = pct(0.50);
    o->p99_ms = pct(0.99);
    double sum = 0;
    for (double x : l) sum += x;
    o->mean_ms = sum / (double)l.size();
    o->max_ms = l.back();
  }
  double busy = s->busy_s + (s->busy_since >= 0 ? now_s() - s->busy_since : 0.0);
  o->busy_s = busy;
  o->rays_per_s = busy > 0 ? (double)s->pixels_done / busy : 0.0;
  o->samples = s->samples_done;
  o->samples_per_s = busy > 0 ? (double)s->samples_done / busy : 0.0;
  note_queue(s);
  o->queued_max = s->q_max;
  o->queued_mean = s->q_last > s->q_since ? s->q_area / (s->q_last - s->q_since) : 0.0;
  o->resident_bytes = s->resident_bytes;
  return VR_OK;
}

vr_status vr_serve_stats_reset(vr_server *s) {
  if (!s) return fail(VR_E_INVALID_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  s->n_submitted = s->n_admitted = s->n_completed = s->n_rejected = s->n_launches = s->n_items = 0;
  s->latencies_ms.clear();
  s->busy_s = 0;
  if (s->busy_since >= 0) s->busy_since = now_s();
  s->pixels_done = 0;
  s->samples_done = 0;
  s->hbm_peak = s->hbm_used;
  s->q_area = 0;
  s->q_since = s->q_last = now_s();
  s->q_max = s->queue.size();
  return VR_OK;
}

vr_status vr_serve_destroy(vr_server *s) {
  if (!s) return fail(VR_E_INVALID_ARG, "server is NULL");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    for (uint64_t t : s->queue) {
      Request &r = *s->requests[t];
      r.state = RState::Cancelled;
      s->volumes[r.volume_id].users--;
    }
    note_queue(s);
    s->queue.clear();
    s->cv_work.notify_all();
  }
  if (s->thread.joinable()) s->thread.join();
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->cv_ooc.notify_all();
  }
  if (s->ooc_thread.joinable()) s->ooc_thread.join();
  (void)s->ops->set_device(s->cfg.device);
  for (Batch &b : s->batches) {
    if (b.stream) (void)s->ops->stream_sync(b.stream);
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    for (Batch &b : s->batches)
      if (b.busy) retire(s, b);
    for (uint64_t t : s->admitted) {
      Request &r = *s->requests[t];
      r.state = RState::Cancelled;
    }
    s->admitted.clear();
    s->cv_done.notify_all();
  }
  {
    // let every waiter observe its final state before the server goes away
    std::unique_lock<std::mutex> lk(s->mu);
    s->cv_done.wait(lk, [&] { return s->waiters == 0; });
  }
  free_server_resources(s);
  delete s;
  return VR_OK;
}

}  // extern "C"
