// device_state.hip -- per-device state the library keeps in the code object
// itself (no allocation): the status word in which kernels record an invalid
// transfer-function table, and the scratch array of vr_render_noalloc.
//
// A table on the device cannot be checked on the host without waiting for
// the device, so the kernels check it while staging it in LDS (load_tf):
// an invalid node (a non-finite channel or a negative extinction) makes the
// call write NaN results, and the word below is set.  vr_device_status waits
// for a stream, then reports and clears it.
#include <mutex>

#include "vr.h"
#include "vr_internal.h"

namespace vr {

__device__ uint32_t g_tf_status;

// Scratch of vr_render_noalloc: the workgroup order of one launch with its
// work-queue counters (the first kScratchOrderInts words) and the block grid's
// occupancy planes (the rest).
// Each GPU holds its own copy until the process ends.  Host code uses it only
// through the per-device address hipGetSymbolAddress returns (the array's
// name on the host is a stand-in, not a device address).
constexpr int64_t kScratchOrderInts = (1 << 18) + kOrderQueueInts;  // 262,144 super-tiles per launch
constexpr size_t kScratchBytes = (1u << 20) + (size_t)kScratchOrderInts * 4;  // 1 MiB of occupancy planes
constexpr size_t kScratchOccBytes = kScratchBytes - (size_t)kScratchOrderInts * 4;
static __device__ __align__(256) uint32_t scratch[kScratchBytes / 4];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint32_t *g_status_addr[kMaxDevices];
bool g_status_done[kMaxDevices];
uint32_t *g_scratch_addr[kMaxDevices];
bool g_scratch_done[kMaxDevices];
}  // namespace

// Device address of the current device's scratch array (set-up once per
// device, with that device current), nullptr on failure.
static uint32_t *scratch_address(int dev) {
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch_done[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) == hipSuccess)
      g_scratch_addr[dev] = static_cast<uint32_t *>(p);
    else
      (void)hipGetLastError();
    g_scratch_done[dev] = true;
  }
  return g_scratch_addr[dev];
}

uint32_t *tf_status_word() {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_status_done[dev]) {
    void *p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(g_tf_status)) == hipSuccess)
      g_status_addr[dev] = static_cast<uint32_t *>(p);
    else
      (void)hipGetLastError();
    g_status_done[dev] = true;
  }
  return g_status_addr[dev];
}

}  // namespace vr

using namespace vr;

extern "C" vr_status vr_device_status(void *stream) {
  uint32_t *w = tf_status_word();
  if (!w) return fail(VR_E_DEVICE, "no device status word on the current device");
  hipError_t e = hipStreamSynchronize((hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "vr_device_status: stream");
  uint32_t v = 0;
  if ((e = hipMemcpy(&v, w, sizeof(v), hipMemcpyDeviceToHost)) != hipSuccess) return hip_fail(e, "vr_device_status: read");
  if (v) {
    const uint32_t zero = 0;
    if ((e = hipMemcpy(w, &zero, sizeof(zero), hipMemcpyHostToDevice)) != hipSuccess)
      return hip_fail(e, "vr_device_status: clear");
    return fail(VR_E_INVALID_ARG,
                "a transfer function read on this device held a non-finite value or a negative extinction; the calls "
                "that read it wrote NaN results");
  }
  return VR_OK;
}

extern "C" vr_status vr_render_noalloc(const vr_volume *vol, const vr_blocks *blocks, const vr_camera *cams,
                                       int32_t n_cams, const vr_tf *tf, const vr_params *p, float *out_rgba,
                                       void *stream) {
  RenderArgs a;
  vr_status s = prepare_render(vol, blocks, cams, n_cams, tf, p, &a);
  if (s) return s;
  if (!out_rgba) return fail(VR_E_INVALID_ARG, "out_rgba is NULL");
  const int64_t tiles = (int64_t)((a.W + kSuperEdge - 1) / kSuperEdge) * ((a.H + kSuperEdge - 1) / kSuperEdge);
  if (tiles > kScratchOrderInts - kOrderQueueInts)
    return fail(VR_E_INVALID_ARG,
                "vr_render_noalloc: a %dx%d view has %lld 16x16 tiles; its scratch orders at most %lld per launch",
                a.W, a.H, (long long)tiles, (long long)(kScratchOrderInts - kOrderQueueInts));
  if (a.mc.skip && occupancy_bytes(a.vol) > kScratchOccBytes)
    return fail(VR_E_INVALID_ARG,
                "vr_render_noalloc: %lld blocks need %zu bytes of occupancy planes; its scratch holds %zu",
                (long long)a.vol.nbx * a.vol.nby * a.vol.nbz, occupancy_bytes(a.vol), kScratchOccBytes);
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "vr_render_noalloc: hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(VR_E_UNSUPPORTED, "vr_render_noalloc: device %d", dev);
  uint32_t *base = scratch_address(dev);
  if (!base) return fail(VR_E_DEVICE, "vr_render_noalloc: no scratch address on device %d", dev);
  RenderScratch sc;
  sc.order = reinterpret_cast<int32_t *>(base);
  sc.order_ints = kScratchOrderInts;
  sc.occ = base + kScratchOrderInts;
  sc.occ_bytes = kScratchOccBytes;
  return render_views(a, cams, n_cams, out_rgba, stream, nullptr, &sc);
}
