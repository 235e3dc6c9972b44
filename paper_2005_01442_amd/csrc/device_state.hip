// device_state.hip -- per-device state the library keeps in the code object
// itself (no allocation): the status word in which kernels record an invalid
// transfer-function table.
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

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint32_t *g_status_addr[kMaxDevices];
bool g_status_done[kMaxDevices];
}  // namespace

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
