/*
 * vr_timeline.h -- diagnostics of the whole-image kernels: a record per
 * wavefront item of the last launch of the forward (k_render) or the adjoint
 * (k_render_bwd), kept only by a library built with VR_TIMELINE defined
 * (python -m paper_2005_01442_amd.timeline builds and reads one).  The
 * product library keeps no records: every call returns VR_E_UNSUPPORTED.
 */
#ifndef VR_TIMELINE_H
#define VR_TIMELINE_H

#include <stdint.h>

#include "vr.h"

#ifdef __cplusplus
extern "C" {
#endif

enum { VR_TIMELINE_FORWARD = 0, VR_TIMELINE_ADJOINT = 1 };

/* Copy the records of the last launch of `kernel` (VR_TIMELINE_*) into
 * host_out (HOST, caller-owned, 4 uint64 per record, at most max_records
 * records) and store the launch's record count in *n_records (HOST).  Record
 * w (wavefront w % 4 of workgroup item w / 4, whichever resident wavefront of
 * a queued launch took it): start and end of the item on the 100 MHz constant
 * clock (s_memrealtime), then (super-tile index << 32 | hardware id of the
 * wavefront that ran it: SE, CU, SIMD, wave slot fields of HW_ID), then the
 * item's work (forward: evaluated samples; adjoint: lattice samples of its
 * rays).  Synchronises the device first.  Launches beyond 131072 items keep
 * their first 131072.  Errors: VR_E_UNSUPPORTED (built
 * without VR_TIMELINE), VR_E_INVALID_ARG (unknown kernel, null pointers),
 * VR_E_DEVICE. */
vr_status vr_timeline_read(int32_t kernel, uint64_t *host_out, uint64_t max_records, uint64_t *n_records);

#ifdef __cplusplus
}
#endif

#endif /* VR_TIMELINE_H */
