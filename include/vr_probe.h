/*
 * vr_probe.h -- measurement primitive of the ray caster's benchmark: a plain
 * streaming read of device memory, the achievable HBM read bandwidth that
 * the renderer's traffic is compared against.  Not part of the rendering
 * path.
 */
#ifndef VR_PROBE_H
#define VR_PROBE_H

#include <stdint.h>

#include "vr.h"

#ifdef __cplusplus
extern "C" {
#endif

/* Read `bytes` of device memory at `buf` once, with 16-byte loads spread over
 * every compute unit (each lane keeps four loads in flight), and fold the
 * data into *sink (XOR, so the loads cannot be dropped).
 * buf: DEVICE, 16-byte aligned; bytes: a positive multiple of 16.
 * sink: DEVICE, one uint32_t, caller-owned (its value is meaningless; the
 * caller zeroes it or not).  Enqueued on `stream`; time it with events.
 * Errors: VR_E_INVALID_ARG (null pointers, misalignment, bytes not a positive
 * multiple of 16), VR_E_DEVICE. */
vr_status vr_probe_stream_read(const void *buf, uint64_t bytes, uint32_t *sink, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* VR_PROBE_H */
