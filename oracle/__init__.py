"""FP64 CPU oracle for tricubic direct volume ray casting.

TEST INFRASTRUCTURE ONLY: the test suite, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import this package; the GPU library and
its Python binding never do.  It shares no code with the GPU path; only the
seeded inputs of ``synth`` feed both.

Scalar parameters that the GPU ABI carries in fp32 (step, early-termination
threshold, TF value range) are rounded to fp32 here before the FP64
arithmetic, so both sides march the same lattice.

The arithmetic lives in ``oracle.c`` (plain scalar C, FP64, OpenMP over
pixels); ``brute.py`` is an independent pure-Python brute force for tiny
volumes.  This module only marshals NumPy arrays into the C calls.

Parity notes:
  * every function here is pinned by the ``-m "not gpu"`` tests in
    ``tests/test_oracle_*.py`` (closed forms, invariants, brute force).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

DTYPES = {np.dtype(np.uint16): 0, np.dtype(np.int16): 1, np.dtype(np.float32): 2, np.dtype(np.float64): 3}


def build(force: bool = True) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` with gcc (no FMA contraction,
    no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        cmd = [
            "gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-ffp-contract=off",
            "-Wall", "-Wno-unknown-pragmas", "-o", _LIB_PATH + ".tmp", _SRC, "-lm",
        ]
        subprocess.run(cmd, check=True)
        os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


_lib = None


def load(path: str):
    """Load an oracle shared library from ``path`` with its prototypes."""
    L = ctypes.CDLL(path)
    _prototypes(L)
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = load(_LIB_PATH)
    return _lib


def use(library):
    """Make ``library`` (a handle from ``load``) the one every call goes
    through; returns the previous one.  Used by the mutation tests."""
    global _lib
    prev = _lib
    _lib = library
    return prev


def _prototypes(L):
    if True:
        P = ctypes.c_void_p
        i64 = ctypes.c_long
        i32 = ctypes.c_int
        f64 = ctypes.c_double
        f32 = ctypes.c_float
        L.oracle_num_threads.restype = i32
        L.oracle_set_num_threads.argtypes = [i32]
        L.oracle_set_num_threads.restype = None
        L.oracle_blocks.argtypes = [P, i32, i64, i64, i64, i32, P]
        L.oracle_blocks.restype = i32
        L.oracle_occupancy.argtypes = [P, i64, P, i32, f32, f32, f32, P]
        L.oracle_occupancy.restype = i32
        L.oracle_render.argtypes = [P, i32, i64, i64, i64, P, i32, i32, i32, P, i32, f64, f64, f64, f64,
                                    P, i32, i32, P, i64, P, P, P]
        L.oracle_render.restype = i32
        L.oracle_grad.argtypes = [P, i32, i64, i64, i64, P, i32, i32, i32, P, i32, f64, f64, f64, f64,
                                  P, i32, P, P, P, P, P]
        L.oracle_grad.restype = i32
        L.oracle_ray.argtypes = [P, i32, i32, i64, i64, i64, i64, i64, f64, P, P]
        L.oracle_ray.restype = i32
        L.oracle_sample.argtypes = [P, i32, i64, i64, i64, f64, f64, f64]
        L.oracle_sample.restype = f64
        L.oracle_weights.argtypes = [f64, P]
        L.oracle_weights.restype = None
        L.oracle_lattice.argtypes = [P, i32, i32, i32, i64, i64, i64, f64, P]
        L.oracle_lattice.restype = i32
        L.oracle_render_shaded.argtypes = [P, i32, i64, i64, i64, P, i32, i32, i32, P, i32, f64, f64, f64, f64,
                                           P, i32, P, P, i64, P, P, P]
        L.oracle_render_shaded.restype = i32
        L.oracle_gradient.argtypes = [P, i32, i64, i64, i64, f64, f64, f64, P]
        L.oracle_gradient.restype = None
        L.oracle_dweights.argtypes = [f64, P]
        L.oracle_dweights.restype = None
        L.oracle_preint_table.argtypes = [P, i32, f64, P]
        L.oracle_preint_table.restype = i32
        L.oracle_render_preint.argtypes = [P, i32, i64, i64, i64, P, i32, i32, i32, P, i32, f64, f64, P, f64, f64,
                                           P, i32, P, i64, P, P, P]
        L.oracle_render_preint.restype = i32
        L.oracle_prefilter.argtypes = [P, i32, i64, i64, i64, P]
        L.oracle_prefilter.restype = i32
        L.oracle_sample_filter.argtypes = [P, i32, i64, i64, i64, f64, f64, f64, i32]
        L.oracle_sample_filter.restype = f64
        L.oracle_catmull_rom.argtypes = [f64, P]
        L.oracle_catmull_rom.restype = None


def f32(x) -> float:
    """The value as the fp32 the GPU ABI carries (step, thresholds, TF range)."""
    return float(np.float32(x))


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _vol(vol):
    vol = np.ascontiguousarray(vol)
    if vol.dtype not in DTYPES:
        raise TypeError(f"unsupported volume dtype {vol.dtype}")
    nz, ny, nx = vol.shape
    return vol, DTYPES[vol.dtype], nx, ny, nz


def pack_cameras(cameras) -> np.ndarray:
    """Pack cameras into the oracle's 16-double rows: projection, eye, right,
    up, forward, fov_y, ortho_w, ortho_h."""
    rows = []
    for c in cameras:
        rows.append(
            [float(c.projection), *map(float, c.eye), *map(float, c.right), *map(float, c.up),
             *map(float, c.forward), float(c.fov_y), float(c.ortho_w), float(c.ortho_h)]
        )
    return np.ascontiguousarray(np.array(rows, dtype=np.float64))


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def set_num_threads(n: int) -> None:
    """Threads the following oracle calls use (n >= 1)."""
    lib().oracle_set_num_threads(int(n))


def blocks(vol, edge: int = 16) -> np.ndarray:
    """Per-block (min, max) over the tricubic footprint; shape (nbz, nby, nbx, 2)."""
    vol, dt, nx, ny, nz = _vol(vol)
    nbx, nby, nbz = -(-nx // edge), -(-ny // edge), -(-nz // edge)
    out = np.zeros((nbz, nby, nbx, 2), dtype=np.float64)
    rc = lib().oracle_blocks(_ptr(vol), dt, nx, ny, nz, edge, _ptr(out))
    if rc:
        raise ValueError("oracle_blocks rejected its arguments")
    return out


CATMULL_ROM_WIDEN = 0.4765625  # ((1 + 2/8)^3 - 1) / 2


def occupancy(minmax, tf, filter=0) -> np.ndarray:
    """One byte per block: 1 when the block can hold a visible sample under tf
    (filter 1, Catmull-Rom: over the widened range of ``oracle_occupancy``)."""
    mm = np.ascontiguousarray(minmax, dtype=np.float64)
    nb = mm.size // 2
    occ = np.zeros(mm.shape[:-1], dtype=np.uint8)
    table = np.ascontiguousarray(tf.table, dtype=np.float32)
    widen = CATMULL_ROM_WIDEN if filter == 1 else 0.0
    rc = lib().oracle_occupancy(_ptr(mm), nb, _ptr(table), table.shape[0], f32(tf.v0), f32(tf.v1), widen, _ptr(occ))
    if rc:
        raise ValueError("oracle_occupancy rejected its arguments")
    return occ


def shade_params(sh) -> np.ndarray:
    """The oracle's 9 lighting doubles (ambient, diffuse, specular, shininess,
    light x, y, z, headlight flag, grad_min) from a mapping or an object with
    those fields; the scalars are rounded to the fp32 the GPU ABI carries."""
    get = (lambda k: sh[k]) if isinstance(sh, dict) else (lambda k: getattr(sh, k))
    light = [f32(x) for x in get("light")]
    return np.array([f32(get("ambient")), f32(get("diffuse")), f32(get("specular")), f32(get("shininess")),
                     *light, 1.0 if get("headlight") else 0.0, f32(get("grad_min"))], dtype=np.float64)


def render(vol, cameras, tf, step, ert=0.0, occ=None, edge=16, pixels=None, shading=None, filter=0):
    """FP64 render.  Returns dict(rgba, flags, counts); rgba is (views, H, W, 4)
    for a full render or (n, 4) for a pixel list.  ``shading`` (see
    ``shade_params``) switches on local lighting; ``filter`` 1 reconstructs
    with Catmull-Rom instead of the cubic B-spline, 2 pre-classifies
    (opacity-weighted B-spline of the classified taps), 3 reconstructs
    trilinearly; all unlit only."""
    vol, dt, nx, ny, nz = _vol(vol)
    cams = pack_cameras(cameras)
    W, H = int(cameras[0].width), int(cameras[0].height)
    table = np.ascontiguousarray(tf.table, dtype=np.float32)
    occ_a = None if occ is None else np.ascontiguousarray(occ, dtype=np.uint8)
    if pixels is None:
        n = len(cameras) * W * H
        pix = None
        shape = (len(cameras), H, W)
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64)
        n = pix.shape[0]
        shape = (n,)
    rgba = np.zeros(shape + (4,), dtype=np.float64)
    flags = np.zeros(shape, dtype=np.uint8)
    counts = np.zeros(shape + (2,), dtype=np.int64)
    if shading is None:
        rc = lib().oracle_render(
            _ptr(vol), dt, nx, ny, nz, _ptr(cams), len(cameras), W, H, _ptr(table), table.shape[0],
            f32(tf.v0), f32(tf.v1), f32(step), f32(ert), _ptr(occ_a), int(edge), int(filter), _ptr(pix), n,
            _ptr(rgba), _ptr(flags), _ptr(counts),
        )
    else:
        if filter != 0:
            raise ValueError("local lighting is defined for the cubic B-spline only")
        sp = shade_params(shading)
        rc = lib().oracle_render_shaded(
            _ptr(vol), dt, nx, ny, nz, _ptr(cams), len(cameras), W, H, _ptr(table), table.shape[0],
            f32(tf.v0), f32(tf.v1), f32(step), f32(ert), _ptr(occ_a), int(edge), _ptr(sp), _ptr(pix), n,
            _ptr(rgba), _ptr(flags), _ptr(counts),
        )
    if rc:
        raise ValueError("oracle_render rejected its arguments")
    return dict(rgba=rgba, flags=flags, counts=counts)


def grad(vol, cameras, tf, step, grad_rgba, ert=0.0, occ=None, edge=16, want_volume=True, want_tf=True,
         magnitudes=False):
    """Gradient of sum(grad_rgba * RGBA) w.r.t. the voxel values and the TF
    table, in FP64.  Returns (grad_volume shaped like vol or None, grad_tf (K, 4)
    or None); with ``magnitudes`` also the same sums taken over the terms'
    magnitudes (the scale of any evaluation's rounding error), as a 4-tuple
    (grad_volume, grad_tf, mag_volume, mag_tf)."""
    vol, dt, nx, ny, nz = _vol(vol)
    cams = pack_cameras(cameras)
    W, H = int(cameras[0].width), int(cameras[0].height)
    table = np.ascontiguousarray(tf.table, dtype=np.float32)
    g = np.ascontiguousarray(grad_rgba, dtype=np.float64).reshape(len(cameras), H, W, 4)
    gv = np.zeros(vol.shape, dtype=np.float64) if want_volume else None
    gt = np.zeros(table.shape, dtype=np.float64) if want_tf else None
    mv = np.zeros(vol.shape, dtype=np.float64) if (want_volume and magnitudes) else None
    mt = np.zeros(table.shape, dtype=np.float64) if (want_tf and magnitudes) else None
    occ_a = None if occ is None else np.ascontiguousarray(occ, dtype=np.uint8)
    rc = lib().oracle_grad(
        _ptr(vol), dt, nx, ny, nz, _ptr(cams), len(cameras), W, H, _ptr(table), table.shape[0],
        f32(tf.v0), f32(tf.v1), f32(step), f32(ert), _ptr(occ_a), int(edge), _ptr(g), _ptr(gv), _ptr(gt),
        _ptr(mv), _ptr(mt),
    )
    if rc:
        raise ValueError("oracle_grad rejected its arguments")
    return (gv, gt, mv, mt) if magnitudes else (gv, gt)


def lattice(cameras, dims_xyz, step) -> np.ndarray:
    """Lattice sample count of every pixel, shape (views, H, W)."""
    cams = pack_cameras(cameras)
    W, H = int(cameras[0].width), int(cameras[0].height)
    out = np.zeros((len(cameras), H, W), dtype=np.int64)
    rc = lib().oracle_lattice(_ptr(cams), len(cameras), W, H, int(dims_xyz[0]), int(dims_xyz[1]),
                              int(dims_xyz[2]), f32(step), _ptr(out))
    if rc:
        raise ValueError("oracle_lattice rejected its arguments")
    return out


def ray(camera, row, col, dims_xyz, step):
    """(origin, direction, t_in, t_out, lattice count, hit) of one pixel's ray."""
    cam = pack_cameras([camera])
    out = np.zeros(8, dtype=np.float64)
    ns = ctypes.c_long(0)
    hit = lib().oracle_ray(_ptr(cam), int(camera.width), int(camera.height), int(row), int(col),
                           int(dims_xyz[0]), int(dims_xyz[1]), int(dims_xyz[2]), f32(step), _ptr(out),
                           ctypes.byref(ns))
    return out[:3].copy(), out[3:6].copy(), float(out[6]), float(out[7]), int(ns.value), bool(hit)


def sample(vol, p, filter=0) -> float:
    """Value of ``vol`` at point p = (x, y, z): cubic B-spline (filter 0),
    Catmull-Rom (1) or trilinear (3)."""
    vol, dt, nx, ny, nz = _vol(vol)
    if filter == 0:
        return float(lib().oracle_sample(_ptr(vol), dt, nx, ny, nz, float(p[0]), float(p[1]), float(p[2])))
    return float(lib().oracle_sample_filter(_ptr(vol), dt, nx, ny, nz, float(p[0]), float(p[1]), float(p[2]),
                                            int(filter)))


def catmull_rom_weights(f) -> np.ndarray:
    w = np.zeros(4, dtype=np.float64)
    lib().oracle_catmull_rom(float(f), _ptr(w))
    return w


def weights(f) -> np.ndarray:
    w = np.zeros(4, dtype=np.float64)
    lib().oracle_weights(float(f), _ptr(w))
    return w


def dweights(f) -> np.ndarray:
    """Derivatives of the four B-spline weights at fractional offset f."""
    d = np.zeros(4, dtype=np.float64)
    lib().oracle_dweights(float(f), _ptr(d))
    return d


def gradient(vol, p) -> np.ndarray:
    """Analytic gradient of the tricubic reconstruction of ``vol`` at p."""
    vol, dt, nx, ny, nz = _vol(vol)
    g = np.zeros(3, dtype=np.float64)
    lib().oracle_gradient(_ptr(vol), dt, nx, ny, nz, float(p[0]), float(p[1]), float(p[2]), _ptr(g))
    return g


def preint_table(tf, step) -> np.ndarray:
    """Pre-integrated segment table (K, K, 4): entry (i, j) = (C_r, C_g, C_b,
    alpha) of a segment of length ``step`` whose value rises linearly from TF
    node i to node j."""
    table = np.ascontiguousarray(tf.table, dtype=np.float32)
    K = table.shape[0]
    out = np.zeros((K, K, 4), dtype=np.float64)
    if lib().oracle_preint_table(_ptr(table), K, f32(step), _ptr(out)):
        raise ValueError("oracle_preint_table rejected its arguments")
    return out


def render_preint(vol, cameras, tf, step, ert=0.0, minmax=None, edge=16, pixels=None, table=None):
    """FP64 pre-integrated render (cells between lattice boundaries, table
    lookup per cell).  ``minmax`` (per-block, from ``blocks``) enables the
    pair-of-blocks skip rule.  Returns dict(rgba, flags, counts) as ``render``."""
    vol, dt, nx, ny, nz = _vol(vol)
    cams = pack_cameras(cameras)
    W, H = int(cameras[0].width), int(cameras[0].height)
    tf_tab = np.ascontiguousarray(tf.table, dtype=np.float32)
    tab = preint_table(tf, step) if table is None else np.ascontiguousarray(table, dtype=np.float64)
    mm = None if minmax is None else np.ascontiguousarray(minmax, dtype=np.float64)
    if pixels is None:
        n = len(cameras) * W * H
        pix = None
        shape = (len(cameras), H, W)
    else:
        pix = np.ascontiguousarray(pixels, dtype=np.int64)
        n = pix.shape[0]
        shape = (n,)
    rgba = np.zeros(shape + (4,), dtype=np.float64)
    flags = np.zeros(shape, dtype=np.uint8)
    counts = np.zeros(shape + (2,), dtype=np.int64)
    rc = lib().oracle_render_preint(
        _ptr(vol), dt, nx, ny, nz, _ptr(cams), len(cameras), W, H, _ptr(tf_tab), tf_tab.shape[0], f32(tf.v0),
        f32(tf.v1), _ptr(tab), f32(step), f32(ert), _ptr(mm), int(edge), _ptr(pix), n, _ptr(rgba), _ptr(flags),
        _ptr(counts),
    )
    if rc:
        raise ValueError("oracle_render_preint rejected its arguments")
    return dict(rgba=rgba, flags=flags, counts=counts)


def prefilter(vol) -> np.ndarray:
    """Interpolating cubic B-spline coefficients of ``vol`` (FP64, same shape):
    the B-spline of the result passes through every voxel value."""
    vol, dt, nx, ny, nz = _vol(vol)
    out = np.zeros(vol.shape, dtype=np.float64)
    if lib().oracle_prefilter(_ptr(vol), dt, nx, ny, nz, _ptr(out)):
        raise ValueError("oracle_prefilter rejected its arguments")
    return out
