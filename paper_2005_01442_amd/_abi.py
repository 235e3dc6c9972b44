"""ctypes mirror of include/vr.h and the loader of libvr.so.

There is no fallback: if the gfx950 library is missing the import of the
binding raises, naming the build step.
"""

from __future__ import annotations

import ctypes
import os
from ctypes import c_double, c_float, c_int32, c_int64, c_uint64, c_void_p, POINTER

HERE = os.path.dirname(os.path.abspath(__file__))
# VR_LIBRARY names another build of the same library (the diagnostics build
# of paper_2005_01442_amd.timeline); by default the in-tree libvr.so
LIB_PATH = os.environ.get("VR_LIBRARY") or os.path.join(HERE, "libvr.so")

VR_OK = 0
STATUS_NAMES = {
    0: "VR_OK",
    1: "VR_E_INVALID_ARG",
    2: "VR_E_UNSUPPORTED",
    3: "VR_E_OOM",
    4: "VR_E_DEVICE",
    5: "VR_E_BUDGET",
    6: "VR_E_NOT_FOUND",
    7: "VR_E_BUSY",
    8: "VR_E_TIMEOUT",
    9: "VR_E_SHUTDOWN",
}
VR_U16, VR_I16, VR_F32 = 0, 1, 2
VR_FILTER_BSPLINE, VR_FILTER_CATMULL_ROM, VR_FILTER_BSPLINE_PRECLASSIFIED, VR_FILTER_TRILINEAR = 0, 1, 2, 3
VR_MAX_TF_NODES = 1024
VR_ABI_VERSION = 2


class VrError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        self.status_name = STATUS_NAMES.get(status, str(status))
        super().__init__(f"{self.status_name}: {message}")


class vr_volume(ctypes.Structure):
    _fields_ = [("data", c_void_p), ("dtype", c_int32), ("reserved", c_int32),
                ("nx", c_int64), ("ny", c_int64), ("nz", c_int64)]


class vr_camera(ctypes.Structure):
    _fields_ = [("projection", c_int32), ("width", c_int32), ("height", c_int32), ("reserved", c_int32),
                ("eye", c_double * 3), ("right", c_double * 3), ("up", c_double * 3), ("forward", c_double * 3),
                ("fov_y", c_double), ("ortho_w", c_double), ("ortho_h", c_double)]


class vr_tf(ctypes.Structure):
    _fields_ = [("table", c_void_p), ("K", c_int32), ("v0", c_float), ("v1", c_float)]


class vr_params(ctypes.Structure):
    _fields_ = [("step", c_float), ("ert_threshold", c_float), ("use_skip", c_int32), ("filter", c_int32),
                ("counters", c_void_p)]


class vr_shading(ctypes.Structure):
    _fields_ = [("ambient", c_float), ("diffuse", c_float), ("specular", c_float), ("shininess", c_float),
                ("light", c_float * 3), ("headlight", c_int32), ("grad_min", c_float), ("reserved", c_int32)]


class vr_bricked_stats(ctypes.Structure):
    _fields_ = [("passes", c_uint64), ("bricks_total", c_uint64), ("bricks_occupied", c_uint64),
                ("bricks_uploaded", c_uint64), ("bytes_uploaded", c_uint64), ("bricks_resident", c_uint64),
                ("pool_slots", c_uint64), ("brick_bytes", c_uint64)]


class vr_serve_config(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", c_uint64), ("max_inflight", c_int32), ("max_batch_tiles", c_int32),
                ("device", c_int32), ("reserved", c_int32), ("brick_pool_bytes", c_uint64)]


class vr_request(ctypes.Structure):
    _fields_ = [("volume_id", c_int32), ("K", c_int32), ("tf_table_host", c_void_p), ("tf_v0", c_float),
                ("tf_v1", c_float), ("cam", vr_camera), ("step", c_float), ("ert_threshold", c_float),
                ("use_skip", c_int32), ("reserved", c_int32)]


class vr_serve_stats(ctypes.Structure):
    _fields_ = [("submitted", c_uint64), ("admitted", c_uint64), ("completed", c_uint64), ("rejected", c_uint64),
                ("queued", c_uint64), ("inflight", c_uint64), ("hbm_used", c_uint64), ("hbm_peak", c_uint64),
                ("launches", c_uint64), ("tiles", c_uint64), ("p50_ms", c_double), ("p99_ms", c_double),
                ("mean_ms", c_double), ("max_ms", c_double), ("rays_per_s", c_double), ("busy_s", c_double),
                ("samples", c_uint64), ("samples_per_s", c_double), ("queued_max", c_uint64),
                ("queued_mean", c_double), ("resident_bytes", c_uint64)]


# exported function -> (argtypes, restype)
PROTOTYPES = {
    "vr_abi_version": ([], c_int32),
    "vr_last_error": ([], ctypes.c_char_p),
    "vr_build_blocks": ([POINTER(vr_volume), c_int32, c_void_p, POINTER(c_void_p)], c_int32),
    "vr_blocks_info": ([c_void_p, POINTER(c_int64), POINTER(c_int32)], c_int32),
    "vr_blocks_minmax": ([c_void_p, c_void_p, c_int64, c_void_p], c_int32),
    "vr_block_occupancy": ([c_void_p, POINTER(vr_tf), c_void_p, c_int64, c_void_p], c_int32),
    "vr_blocks_free": ([c_void_p], None),
    "vr_render": ([POINTER(vr_volume), c_void_p, POINTER(vr_camera), c_int32, POINTER(vr_tf), POINTER(vr_params),
                   c_void_p, c_void_p], c_int32),
    "vr_render_noalloc": ([POINTER(vr_volume), c_void_p, POINTER(vr_camera), c_int32, POINTER(vr_tf),
                           POINTER(vr_params), c_void_p, c_void_p], c_int32),
    "vr_render_shaded": ([POINTER(vr_volume), c_void_p, POINTER(vr_camera), c_int32, POINTER(vr_tf),
                          POINTER(vr_params), POINTER(vr_shading), c_void_p, c_void_p], c_int32),
    "vr_preint_build": ([POINTER(vr_tf), c_float, c_void_p, POINTER(c_void_p)], c_int32),
    "vr_preint_table": ([c_void_p, c_void_p, c_int64, c_void_p], c_int32),
    "vr_preint_free": ([c_void_p], None),
    "vr_render_preint": ([POINTER(vr_volume), c_void_p, POINTER(vr_camera), c_int32, POINTER(vr_tf),
                          POINTER(vr_params), c_void_p, c_void_p, c_void_p], c_int32),
    "vr_bricked_create": ([POINTER(vr_volume), c_int32, c_uint64, POINTER(c_void_p)], c_int32),
    "vr_bricked_render": ([c_void_p, POINTER(vr_camera), c_int32, POINTER(vr_tf), POINTER(vr_params), c_void_p,
                           c_void_p], c_int32),
    "vr_bricked_stats_get": ([c_void_p, POINTER(vr_bricked_stats)], c_int32),
    "vr_brick_order": ([POINTER(c_int64), c_int32, POINTER(vr_camera), POINTER(c_int64), c_int64], c_int32),
    "vr_bricked_free": ([c_void_p], None),
    "vr_prefilter_bspline": ([POINTER(vr_volume), c_void_p, c_void_p], c_int32),
    "vr_render_backward": ([POINTER(vr_volume), c_void_p, POINTER(vr_camera), c_int32, POINTER(vr_tf),
                            POINTER(vr_params), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p], c_int32),
    "vr_serve_create": ([POINTER(vr_serve_config), POINTER(c_void_p)], c_int32),
    "vr_serve_add_volume": ([c_void_p, POINTER(vr_volume), c_int32, POINTER(c_int32)], c_int32),
    "vr_serve_remove_volume": ([c_void_p, c_int32], c_int32),
    "vr_serve_add_host_volume": ([c_void_p, POINTER(vr_volume), c_int32, POINTER(c_int32)], c_int32),
    "vr_serve_submit": ([c_void_p, POINTER(vr_request), POINTER(c_uint64)], c_int32),
    "vr_serve_wait": ([c_void_p, c_uint64, c_int64, POINTER(c_void_p)], c_int32),
    "vr_serve_release": ([c_void_p, c_uint64], c_int32),
    "vr_serve_stats_get": ([c_void_p, POINTER(vr_serve_stats)], c_int32),
    "vr_serve_stats_reset": ([c_void_p], c_int32),
    "vr_serve_destroy": ([c_void_p], c_int32),
    "vr_device_status": ([c_void_p], c_int32),
    "vr_probe_stream_read": ([c_void_p, c_uint64, c_void_p, c_void_p], c_int32),
    "vr_timeline_read": ([c_int32, c_void_p, c_uint64, POINTER(c_uint64)], c_int32),
    "vr_fallback_counts": ([POINTER(c_uint64), POINTER(c_uint64)], c_int32),
}

_lib = None


def lib():
    """Load libvr.so (built by ``paper_2005_01442_amd.build``); raise if absent."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build the gfx950 HIP library first "
                "(python -m paper_2005_01442_amd.build, or __graft_entry__.build())"
            )
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in PROTOTYPES.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        if L.vr_abi_version() != VR_ABI_VERSION:
            raise RuntimeError("libvr.so ABI version mismatch")
        _lib = L
    return _lib


def check(status):
    if status != VR_OK:
        msg = lib().vr_last_error()
        raise VrError(status, msg.decode() if msg else "")
    return status
