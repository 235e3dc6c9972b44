"""MI355X (gfx950) tricubic volume ray caster: Python binding of libvr.so.

Every function here marshals PyTorch device tensors and camera objects into
the C ABI of ``include/vr.h`` and calls it; all rendering arithmetic runs in
the HIP kernels of ``csrc/``.  PyTorch provides device memory and streams.
The names follow the C ABI (``vr_build_blocks``, ``vr_render``,
``vr_render_backward``, ``vr_serve_*``); ``render`` and ``VolumeRender`` are
conveniences on top of them.

Importing this package loads ``libvr.so`` and raises if it has not been built.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _abi
from ._abi import (VrError, VR_F32, VR_FILTER_BSPLINE, VR_FILTER_BSPLINE_PRECLASSIFIED, VR_FILTER_CATMULL_ROM,  # noqa: F401
                   VR_FILTER_TRILINEAR, VR_I16, VR_U16, check, lib)

__all__ = [
    "VrError",
    "Volume",
    "Blocks",
    "TF",
    "vr_build_blocks",
    "vr_blocks_minmax",
    "vr_block_occupancy",
    "vr_render",
    "vr_render_noalloc",
    "vr_render_backward",
    "device_status",
    "Shading",
    "PreintTable",
    "vr_prefilter_bspline",
    "BrickedVolume",
    "vr_brick_order",
    "vr_preint_build",
    "vr_preint_table",
    "vr_render_preint",
    "render",
    "VolumeRender",
    "Server",
    "vr_serve_create",
    "vr_serve_add_volume",
    "vr_serve_add_host_volume",
    "vr_serve_remove_volume",
    "vr_serve_submit",
    "vr_serve_wait",
    "vr_serve_release",
    "vr_serve_stats_get",
    "vr_serve_stats_reset",
    "vr_serve_destroy",
]

lib()  # fail loudly at import when the HIP library is missing

_TORCH_DTYPES = {torch.int16: VR_I16, torch.float32: VR_F32}
if hasattr(torch, "uint16"):
    _TORCH_DTYPES[torch.uint16] = VR_U16


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


class Volume:
    """A device volume: a CUDA tensor of shape (nz, ny, nx), x fastest.

    ``dtype`` overrides the element type given to the library (use VR_U16
    with an int16 tensor holding unsigned 16-bit data)."""

    def __init__(self, tensor: torch.Tensor, dtype: int | None = None):
        if not tensor.is_cuda:
            raise ValueError("volume tensor must be on the GPU")
        if tensor.dim() != 3 or not tensor.is_contiguous():
            raise ValueError("volume tensor must be contiguous with shape (nz, ny, nx)")
        if dtype is None:
            if tensor.dtype not in _TORCH_DTYPES:
                raise TypeError(f"unsupported volume dtype {tensor.dtype}")
            dtype = _TORCH_DTYPES[tensor.dtype]
        self.tensor = tensor
        self.dtype = dtype
        nz, ny, nx = tensor.shape
        self.dims = (int(nx), int(ny), int(nz))
        self.c = _abi.vr_volume(tensor.data_ptr(), dtype, 0, nx, ny, nz)


class TF:
    """A device transfer-function table (K, 4) fp32 with its value range."""

    def __init__(self, table: torch.Tensor, v0: float, v1: float):
        if not table.is_cuda or table.dtype != torch.float32 or table.dim() != 2 or table.shape[1] != 4:
            raise ValueError("TF table must be a (K, 4) float32 CUDA tensor")
        self.table = table.contiguous()
        self.v0 = float(v0)
        self.v1 = float(v1)
        self.c = _abi.vr_tf(self.table.data_ptr(), int(self.table.shape[0]), self.v0, self.v1)

    @property
    def K(self):
        return int(self.table.shape[0])


def camera_struct(cam) -> _abi.vr_camera:
    c = _abi.vr_camera()
    c.projection = int(cam.projection)
    c.width = int(cam.width)
    c.height = int(cam.height)
    for name in ("eye", "right", "up", "forward"):
        arr = getattr(c, name)
        src = getattr(cam, name)
        for k in range(3):
            arr[k] = float(src[k])
    c.fov_y = float(cam.fov_y)
    c.ortho_w = float(cam.ortho_w)
    c.ortho_h = float(cam.ortho_h)
    return c


def _cameras(cams):
    """ctypes array of the cameras; None for an empty list (the library then
    rejects the call with VR_E_INVALID_ARG)."""
    if len(cams) == 0:
        return None
    arr = (_abi.vr_camera * len(cams))()
    for i, cam in enumerate(cams):
        arr[i] = camera_struct(cam)
    return arr


def _image_size(cams):
    """(W, H) of the views; (0, 0) for an empty list."""
    return (int(cams[0].width), int(cams[0].height)) if len(cams) else (0, 0)


class Blocks:
    """Library-owned block min/max structure of one volume."""

    def __init__(self, ptr, volume: Volume):
        self.ptr = ptr
        self.volume = volume  # keeps the volume memory alive
        dims = (ctypes.c_int64 * 3)()
        edge = ctypes.c_int32(0)
        check(lib().vr_blocks_info(ptr, dims, ctypes.byref(edge)))
        self.grid = (int(dims[0]), int(dims[1]), int(dims[2]))
        self.edge = int(edge.value)

    @property
    def count(self):
        return self.grid[0] * self.grid[1] * self.grid[2]

    def __del__(self):
        if getattr(self, "ptr", None):
            try:
                lib().vr_blocks_free(self.ptr)
            except Exception:
                pass
            self.ptr = None


def vr_build_blocks(volume: Volume, block_edge: int = 16, stream=None) -> Blocks:
    out = ctypes.c_void_p()
    check(lib().vr_build_blocks(ctypes.byref(volume.c), int(block_edge), _stream_ptr(stream), ctypes.byref(out)))
    return Blocks(out, volume)


def vr_blocks_minmax(blocks: Blocks, stream=None) -> torch.Tensor:
    nbx, nby, nbz = blocks.grid
    dst = torch.empty((nbz, nby, nbx, 2), dtype=torch.float32, device=blocks.volume.tensor.device)
    check(lib().vr_blocks_minmax(blocks.ptr, ctypes.c_void_p(dst.data_ptr()), dst.numel(), _stream_ptr(stream)))
    return dst


def vr_block_occupancy(blocks: Blocks, tf: TF, stream=None) -> torch.Tensor:
    nbx, nby, nbz = blocks.grid
    dst = torch.empty((nbz, nby, nbx), dtype=torch.uint8, device=blocks.volume.tensor.device)
    check(lib().vr_block_occupancy(blocks.ptr, ctypes.byref(tf.c), ctypes.c_void_p(dst.data_ptr()), dst.numel(),
                                   _stream_ptr(stream)))
    return dst


def _params(step, ert, use_skip, counters, filter=0):
    p = _abi.vr_params()
    p.step = float(step)
    p.ert_threshold = float(ert)
    p.use_skip = 1 if use_skip else 0
    p.filter = int(filter)
    p.counters = None if counters is None else counters.data_ptr()
    return p


@dataclass
class Shading:
    """Local lighting of ``vr_render_shaded``: every sample's colour c becomes
    c (ambient + diffuse |n.L|) + specular |n.H|^shininess with the normal n
    from the gradient of the cubic reconstruction (two-sided Blinn-Phong)."""

    ambient: float = 0.3
    diffuse: float = 0.7
    specular: float = 0.3
    shininess: float = 16.0
    light: tuple = (0.0, 0.0, -1.0)
    headlight: bool = True
    grad_min: float = 1.0

    def struct(self) -> _abi.vr_shading:
        c = _abi.vr_shading()
        c.ambient, c.diffuse, c.specular, c.shininess = (float(self.ambient), float(self.diffuse),
                                                         float(self.specular), float(self.shininess))
        for a in range(3):
            c.light[a] = float(self.light[a])
        c.headlight = 1 if self.headlight else 0
        c.grad_min = float(self.grad_min)
        return c


def device_status(stream=None):
    """Wait for ``stream`` and raise VrError (VR_E_INVALID_ARG) if a kernel on
    the current device has met an invalid TF table since the last check
    (``vr_device_status``; the calls that read it wrote NaN results)."""
    check(lib().vr_device_status(_stream_ptr(stream)))


def fallback_counts():
    """(occupancy, order): renders that ran a slower path because a per-call
    buffer could not be allocated or built (``vr_fallback_counts``)."""
    occ, order = ctypes.c_uint64(0), ctypes.c_uint64(0)
    check(lib().vr_fallback_counts(ctypes.byref(occ), ctypes.byref(order)))
    return int(occ.value), int(order.value)


def vr_probe_stream_read(buf: torch.Tensor, sink: torch.Tensor, stream=None):
    """Stream-read the whole of the contiguous CUDA tensor ``buf`` once with
    16-byte loads, folding it into ``sink`` (an int32 CUDA tensor of one
    element): the achievable-HBM-bandwidth probe (time it with events)."""
    if not buf.is_cuda or not buf.is_contiguous() or not sink.is_cuda or sink.dtype != torch.int32:
        raise ValueError("buf must be a contiguous CUDA tensor and sink an int32 CUDA tensor")
    nbytes = buf.numel() * buf.element_size()
    check(lib().vr_probe_stream_read(ctypes.c_void_p(buf.data_ptr()), nbytes, ctypes.c_void_p(sink.data_ptr()),
                                     _stream_ptr(stream)))


def vr_render(volume: Volume, blocks, cameras, tf: TF, step: float, ert: float = 0.0, use_skip: bool = False,
              out: torch.Tensor | None = None, counters: torch.Tensor | None = None, stream=None,
              shading: Shading | None = None, filter: int = 0) -> torch.Tensor:
    """Render len(cameras) views; returns (views, H, W, 4) fp32 premultiplied RGBA.
    ``counters``: optional int64 CUDA tensor of 4 that the kernel adds
    [evaluated samples, lattice samples, rays with samples, samples read from
    global memory instead of an LDS box] to.  ``shading`` switches on local
    lighting (``vr_render_shaded``); ``filter`` selects the reconstruction
    (VR_FILTER_BSPLINE, VR_FILTER_CATMULL_ROM)."""
    W, H = _image_size(cameras)
    if out is None:
        out = torch.empty((len(cameras), H, W, 4), dtype=torch.float32, device=volume.tensor.device)
    if counters is not None and (counters.dtype != torch.int64 or counters.numel() < 4 or not counters.is_cuda):
        raise ValueError("counters must be an int64 CUDA tensor of at least 4 elements")
    cams = _cameras(cameras)
    p = _params(step, ert, use_skip, counters, filter)
    if shading is None:
        check(lib().vr_render(ctypes.byref(volume.c), None if blocks is None else blocks.ptr, cams, len(cameras),
                              ctypes.byref(tf.c), ctypes.byref(p), ctypes.c_void_p(out.data_ptr()),
                              _stream_ptr(stream)))
    else:
        sh = shading.struct()
        check(lib().vr_render_shaded(ctypes.byref(volume.c), None if blocks is None else blocks.ptr, cams,
                                     len(cameras), ctypes.byref(tf.c), ctypes.byref(p), ctypes.byref(sh),
                                     ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def vr_render_noalloc(volume: Volume, blocks, cameras, tf: TF, step: float, ert: float, use_skip: bool,
                      out: torch.Tensor, counters: torch.Tensor | None = None, stream=None, filter: int = 0):
    """vr_render into the caller's ``out`` ((views, H, W, 4) fp32 CUDA tensor)
    without any device allocation (``vr_render_noalloc``: the library's
    per-GPU scratch array holds the launch order and occupancy planes)."""
    if counters is not None and (counters.dtype != torch.int64 or counters.numel() < 4 or not counters.is_cuda):
        raise ValueError("counters must be an int64 CUDA tensor of at least 4 elements")
    W, H = _image_size(cameras)
    if (not out.is_cuda or out.dtype != torch.float32 or not out.is_contiguous()
            or out.numel() < len(cameras) * H * W * 4):
        raise ValueError("out must be a contiguous float32 CUDA tensor holding views x H x W x 4")
    cams = _cameras(cameras)
    p = _params(step, ert, use_skip, counters, filter)
    check(lib().vr_render_noalloc(ctypes.byref(volume.c), None if blocks is None else blocks.ptr, cams, len(cameras),
                                  ctypes.byref(tf.c), ctypes.byref(p), ctypes.c_void_p(out.data_ptr()),
                                  _stream_ptr(stream)))
    return out


def vr_prefilter_bspline(volume: Volume, stream=None) -> Volume:
    """Interpolating cubic B-spline coefficients of ``volume`` as a new fp32
    Volume (render it with ``vr_render`` for an interpolating filter)."""
    out = torch.empty(volume.tensor.shape, dtype=torch.float32, device=volume.tensor.device)
    check(lib().vr_prefilter_bspline(ctypes.byref(volume.c), ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return Volume(out)


class PreintTable:
    """Library-owned pre-integrated segment table of one TF and step."""

    def __init__(self, ptr, tf: TF, step: float):
        self.ptr = ptr
        self.tf = tf  # keeps the TF table memory alive
        self.step = float(step)

    def __del__(self):
        if getattr(self, "ptr", None):
            try:
                lib().vr_preint_free(self.ptr)
            except Exception:
                pass
            self.ptr = None


def vr_preint_build(tf: TF, step: float, stream=None) -> PreintTable:
    out = ctypes.c_void_p()
    check(lib().vr_preint_build(ctypes.byref(tf.c), float(step), _stream_ptr(stream), ctypes.byref(out)))
    return PreintTable(out, tf, step)


def vr_preint_table(table: PreintTable, stream=None) -> torch.Tensor:
    """(K, K, 4) fp32 copy of the table: entry (i, j) = (C_r, C_g, C_b, alpha)."""
    K = table.tf.K
    dst = torch.empty((K, K, 4), dtype=torch.float32, device=table.tf.table.device)
    check(lib().vr_preint_table(table.ptr, ctypes.c_void_p(dst.data_ptr()), dst.numel(), _stream_ptr(stream)))
    return dst


def vr_render_preint(volume: Volume, blocks, cameras, tf: TF, table: PreintTable, step: float, ert: float = 0.0,
                     use_skip: bool = False, out: torch.Tensor | None = None, counters: torch.Tensor | None = None,
                     stream=None) -> torch.Tensor:
    """Pre-integrated render of len(cameras) views; (views, H, W, 4) fp32
    premultiplied RGBA.  ``counters`` as vr_render, counting lattice cells."""
    W, H = _image_size(cameras)
    if out is None:
        out = torch.empty((len(cameras), H, W, 4), dtype=torch.float32, device=volume.tensor.device)
    if counters is not None and (counters.dtype != torch.int64 or counters.numel() < 4 or not counters.is_cuda):
        raise ValueError("counters must be an int64 CUDA tensor of at least 4 elements")
    cams = _cameras(cameras)
    p = _params(step, ert, use_skip, counters)
    check(lib().vr_render_preint(ctypes.byref(volume.c), None if blocks is None else blocks.ptr, cams, len(cameras),
                                 ctypes.byref(tf.c), ctypes.byref(p), table.ptr, ctypes.c_void_p(out.data_ptr()),
                                 _stream_ptr(stream)))
    return out


_NP_DTYPES = {"uint16": VR_U16, "int16": VR_I16, "float32": VR_F32}


class BrickedVolume:
    """A volume kept in pinned host memory as bricks, rendered through a
    device brick pool of ``pool_bytes`` (``vr_bricked_*``).  ``host_array`` is
    a C-contiguous NumPy array (nz, ny, nx) of uint16, int16 or float32, copied
    at construction."""

    def __init__(self, host_array, brick_edge: int = 64, pool_bytes: int = 1 << 30):
        import numpy as np

        arr = np.ascontiguousarray(host_array)
        if str(arr.dtype) not in _NP_DTYPES or arr.ndim != 3:
            raise ValueError("host_array must be a 3-D uint16, int16 or float32 array")
        nz, ny, nx = arr.shape
        hv = _abi.vr_volume(arr.ctypes.data, _NP_DTYPES[str(arr.dtype)], 0, nx, ny, nz)
        out = ctypes.c_void_p()
        check(lib().vr_bricked_create(ctypes.byref(hv), int(brick_edge), int(pool_bytes), ctypes.byref(out)))
        self.ptr = out
        self.shape = arr.shape
        self.brick_edge = int(brick_edge)

    def render(self, cameras, tf: TF, step: float, ert: float = 0.0, out: torch.Tensor | None = None,
               stream=None) -> torch.Tensor:
        W, H = _image_size(cameras)
        if out is None:
            out = torch.empty((len(cameras), H, W, 4), dtype=torch.float32, device=tf.table.device)
        cams = _cameras(cameras)
        p = _params(step, ert, True, None)
        check(lib().vr_bricked_render(self.ptr, cams, len(cameras), ctypes.byref(tf.c), ctypes.byref(p),
                                      ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
        return out

    def stats(self) -> dict:
        st = _abi.vr_bricked_stats()
        check(lib().vr_bricked_stats_get(self.ptr, ctypes.byref(st)))
        return {name: int(getattr(st, name)) for name, _ in st._fields_}

    def __del__(self):
        if getattr(self, "ptr", None):
            try:
                lib().vr_bricked_free(self.ptr)
            except Exception:
                pass
            self.ptr = None


def vr_brick_order(dims_xyz, brick_edge: int, camera):
    """Front-to-back brick order (host only): brick indices, x fastest."""
    import numpy as np

    nb = 1
    for d in dims_xyz:
        nb *= -(-int(d) // int(brick_edge))
    dims = (ctypes.c_int64 * 3)(*[int(d) for d in dims_xyz])
    out = np.zeros(nb, dtype=np.int64)
    cam = camera_struct(camera)
    check(lib().vr_brick_order(dims, int(brick_edge), ctypes.byref(cam),
                               out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), nb))
    return out


def vr_render_backward(volume: Volume, blocks, cameras, tf: TF, step: float, ert: float, use_skip: bool,
                       out_rgba: torch.Tensor, grad_rgba: torch.Tensor, want_volume: bool = True,
                       want_tf: bool = True, stream=None):
    """Gradients (grad_volume (nz, ny, nx) fp32 or None, grad_tf (K, 4) or None)."""
    dev = volume.tensor.device
    gv = torch.empty(volume.tensor.shape, dtype=torch.float32, device=dev) if want_volume else None
    gt = torch.empty((tf.K, 4), dtype=torch.float32, device=dev) if want_tf else None
    grad_rgba = grad_rgba.contiguous()
    cams = _cameras(cameras)
    p = _params(step, ert, use_skip, None)
    check(lib().vr_render_backward(
        ctypes.byref(volume.c), None if blocks is None else blocks.ptr, cams, len(cameras), ctypes.byref(tf.c),
        ctypes.byref(p), ctypes.c_void_p(out_rgba.data_ptr()), ctypes.c_void_p(grad_rgba.data_ptr()),
        None if gv is None else ctypes.c_void_p(gv.data_ptr()), None if gt is None else ctypes.c_void_p(gt.data_ptr()),
        _stream_ptr(stream)))
    return gv, gt


def render(volume_tensor, cameras, tf_table, v0, v1, step, ert=0.0, use_skip=False, blocks=None, block_edge=16):
    """Convenience: tensors in, RGBA tensor out (builds blocks when needed)."""
    vol = volume_tensor if isinstance(volume_tensor, Volume) else Volume(volume_tensor)
    tf = TF(tf_table, v0, v1)
    if use_skip and blocks is None:
        blocks = vr_build_blocks(vol, block_edge)
    return vr_render(vol, blocks, cameras, tf, step, ert, use_skip)


class VolumeRender(torch.autograd.Function):
    """Differentiable render: forward = vr_render, backward = vr_render_backward.

    Saves the inputs and the output image only; per-ray state is recomputed
    in the backward kernel.  The grid must be a float32 CUDA tensor."""

    @staticmethod
    def forward(ctx, grid, tf_table, cameras, v0, v1, step, ert=0.0):
        vol = Volume(grid.detach().contiguous())
        tf = TF(tf_table.detach().contiguous(), v0, v1)
        out = vr_render(vol, None, cameras, tf, step, ert, False)
        ctx.save_for_backward(grid, tf_table, out)
        ctx.cameras, ctx.v0, ctx.v1, ctx.step, ctx.ert = cameras, v0, v1, step, ert
        return out

    @staticmethod
    def backward(ctx, grad_out):
        grid, tf_table, out = ctx.saved_tensors
        vol = Volume(grid.detach().contiguous())
        tf = TF(tf_table.detach().contiguous(), ctx.v0, ctx.v1)
        gv, gt = vr_render_backward(vol, None, ctx.cameras, tf, ctx.step, ctx.ert, False, out, grad_out,
                                    want_volume=ctx.needs_input_grad[0], want_tf=ctx.needs_input_grad[1])
        return gv, gt, None, None, None, None, None


# ------------------------------------------------------------------ serving --

def _request_struct(volume_id, cam, tf_table_np, v0, v1, step, ert, use_skip):
    r = _abi.vr_request()
    r.volume_id = int(volume_id)
    r.K = int(tf_table_np.shape[0])
    r.tf_table_host = tf_table_np.ctypes.data
    r.tf_v0 = float(v0)
    r.tf_v1 = float(v1)
    r.cam = camera_struct(cam)
    r.step = float(step)
    r.ert_threshold = float(ert)
    r.use_skip = 1 if use_skip else 0
    return r


def vr_serve_create(hbm_budget_bytes=4 << 30, max_inflight=32, max_batch_tiles=0, device=0, brick_pool_bytes=0):
    cfg = _abi.vr_serve_config(int(hbm_budget_bytes), int(max_inflight), int(max_batch_tiles), int(device), 0,
                               int(brick_pool_bytes))
    out = ctypes.c_void_p()
    check(lib().vr_serve_create(ctypes.byref(cfg), ctypes.byref(out)))
    return out


def vr_serve_add_volume(server, volume: Volume, block_edge=16):
    vid = ctypes.c_int32(-1)
    check(lib().vr_serve_add_volume(server, ctypes.byref(volume.c), int(block_edge), ctypes.byref(vid)))
    return int(vid.value)


def vr_serve_add_host_volume(server, host_array, brick_edge=64):
    """Register a host (NumPy, (nz, ny, nx) uint16/int16/float32) volume as
    out-of-core bricks that take turns in the server's brick pool."""
    import numpy as np

    arr = np.ascontiguousarray(host_array)
    if str(arr.dtype) not in _NP_DTYPES or arr.ndim != 3:
        raise ValueError("host_array must be a 3-D uint16, int16 or float32 array")
    nz, ny, nx = arr.shape
    hv = _abi.vr_volume(arr.ctypes.data, _NP_DTYPES[str(arr.dtype)], 0, nx, ny, nz)
    vid = ctypes.c_int32(-1)
    check(lib().vr_serve_add_host_volume(server, ctypes.byref(hv), int(brick_edge), ctypes.byref(vid)))
    return int(vid.value)


def vr_serve_remove_volume(server, volume_id):
    check(lib().vr_serve_remove_volume(server, int(volume_id)))


def vr_serve_submit(server, volume_id, cam, tf_table_np, v0, v1, step, ert=0.0, use_skip=True):
    import numpy as np

    table = np.ascontiguousarray(tf_table_np, dtype=np.float32)
    req = _request_struct(volume_id, cam, table, v0, v1, step, ert, use_skip)
    ticket = ctypes.c_uint64(0)
    check(lib().vr_serve_submit(server, ctypes.byref(req), ctypes.byref(ticket)))
    return int(ticket.value)


def vr_serve_wait(server, ticket, timeout_us=-1):
    """Returns the device address of the result image (H*W*4 floats)."""
    ptr = ctypes.c_void_p()
    check(lib().vr_serve_wait(server, ctypes.c_uint64(ticket), int(timeout_us), ctypes.byref(ptr)))
    return int(ptr.value)


def vr_serve_release(server, ticket):
    check(lib().vr_serve_release(server, ctypes.c_uint64(ticket)))


def vr_serve_stats_get(server) -> dict:
    st = _abi.vr_serve_stats()
    check(lib().vr_serve_stats_get(server, ctypes.byref(st)))
    return {name: getattr(st, name) for name, _ in st._fields_}


def vr_serve_stats_reset(server):
    check(lib().vr_serve_stats_reset(server))


def vr_serve_destroy(server):
    check(lib().vr_serve_destroy(server))


class Server:
    """Object wrapper of the vr_serve_* calls."""

    def __init__(self, hbm_budget_bytes=4 << 30, max_inflight=32, max_batch_tiles=0, device=0, brick_pool_bytes=0):
        self.handle = vr_serve_create(hbm_budget_bytes, max_inflight, max_batch_tiles, device, brick_pool_bytes)
        self._volumes = {}

    def add_host_volume(self, host_array, brick_edge=64):
        """Out-of-core volume (host bricks through the shared brick pool)."""
        return vr_serve_add_host_volume(self.handle, host_array, brick_edge)

    def add_volume(self, volume: Volume, block_edge=16):
        vid = vr_serve_add_volume(self.handle, volume, block_edge)
        self._volumes[vid] = volume
        return vid

    def remove_volume(self, vid):
        vr_serve_remove_volume(self.handle, vid)
        self._volumes.pop(vid, None)

    def submit(self, volume_id, cam, tf_table_np, v0, v1, step, ert=0.0, use_skip=True):
        return vr_serve_submit(self.handle, volume_id, cam, tf_table_np, v0, v1, step, ert, use_skip)

    def wait(self, ticket, timeout_us=-1):
        return vr_serve_wait(self.handle, ticket, timeout_us)

    def result(self, ticket, height, width, timeout_us=-1) -> torch.Tensor:
        """Wait, copy the device result into a new tensor, release the ticket."""
        ptr = self.wait(ticket, timeout_us)
        out = torch.empty((height, width, 4), dtype=torch.float32, device="cuda")
        nbytes = height * width * 16
        torch.cuda.current_stream().synchronize()
        _copy_device(out.data_ptr(), ptr, nbytes)
        self.release(ticket)
        return out

    def release(self, ticket):
        vr_serve_release(self.handle, ticket)

    def stats(self):
        return vr_serve_stats_get(self.handle)

    def reset_stats(self):
        vr_serve_stats_reset(self.handle)

    def close(self):
        if self.handle is not None:
            vr_serve_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _copy_device(dst_ptr, src_ptr, nbytes):
    """Device-to-device copy of ``nbytes`` through the HIP runtime (the result
    images are library-owned memory without a tensor)."""
    hip = _hip()
    rc = hip.hipMemcpy(ctypes.c_void_p(dst_ptr), ctypes.c_void_p(src_ptr), ctypes.c_size_t(nbytes), 3)
    if rc != 0:
        raise RuntimeError(f"hipMemcpy failed with {rc}")


_hip_lib = None


def _hip():
    global _hip_lib
    if _hip_lib is None:
        _hip_lib = ctypes.CDLL("libamdhip64.so", mode=ctypes.RTLD_GLOBAL)
        _hip_lib.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
        _hip_lib.hipMemcpy.restype = ctypes.c_int
    return _hip_lib
