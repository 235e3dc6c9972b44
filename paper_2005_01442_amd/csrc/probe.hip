// probe.hip -- streaming-read probe: the achievable HBM read bandwidth the
// benchmark compares the renderer's traffic with (include/vr_probe.h).
#include "vr.h"
#include "vr_internal.h"
#include "vr_probe.h"

namespace vr {

constexpr int kProbeThreads = 256;
constexpr int kProbeWgPerCu = 8;
constexpr int kProbeUnroll = 4;

typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(kProbeThreads) void k_stream_read(const u32x4_t *p, uint64_t n, uint32_t *sink) {
  const uint64_t stride = (uint64_t)gridDim.x * kProbeThreads;
  uint64_t i = (uint64_t)blockIdx.x * kProbeThreads + threadIdx.x;
  uint32_t acc = 0;
  for (; i + (kProbeUnroll - 1) * stride < n; i += kProbeUnroll * stride) {
    u32x4_t v[kProbeUnroll];
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) v[u] = __builtin_nontemporal_load(p + i + u * stride);
#pragma unroll
    for (int u = 0; u < kProbeUnroll; ++u) acc ^= v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
  }
  for (; i < n; i += stride) {
    const u32x4_t v = __builtin_nontemporal_load(p + i);
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  for (int off = 32; off > 0; off >>= 1) acc ^= __shfl_xor(acc, off, kWaveSize);
  if ((threadIdx.x % kWaveSize) == 0) atomicXor(sink, acc);
}

}  // namespace vr

using namespace vr;

extern "C" vr_status vr_probe_stream_read(const void *buf, uint64_t bytes, uint32_t *sink, void *stream) {
  if (!buf || !sink) return fail(VR_E_INVALID_ARG, "buffer or sink is NULL");
  if ((reinterpret_cast<uintptr_t>(buf) & 15u) != 0) return fail(VR_E_INVALID_ARG, "buffer must be 16-byte aligned");
  if (bytes == 0 || (bytes & 15u) != 0) return fail(VR_E_INVALID_ARG, "bytes must be a positive multiple of 16");
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return hip_fail(e, "probe device query");
  const unsigned grid = (unsigned)(cus > 0 ? cus * kProbeWgPerCu : 2048);
  hipLaunchKernelGGL(k_stream_read, dim3(grid), dim3(kProbeThreads), 0, (hipStream_t)stream,
                     static_cast<const u32x4_t *>(buf), bytes / 16, sink);
  e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "probe launch");
  return VR_OK;
}
