"""The C-ABI library without a GPU: it loads, exports every function
include/vr.h declares, its ctypes mirror has the C layout, and argument
validation rejects bad calls before anything touches the device."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = sorted(os.path.join(ROOT, "include", f) for f in os.listdir(os.path.join(ROOT, "include"))
                 if f.endswith(".h"))
HEADER = os.path.join(ROOT, "include", "vr.h")
LIB = os.path.join(ROOT, "paper_2005_01442_amd", "libvr.so")


def _declared_functions():
    text = "\n".join(open(h).read() for h in HEADERS)
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vr_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def abi():
    if not os.path.exists(LIB):
        pytest.fail("libvr.so is not built (run __graft_entry__.build())")
    from paper_2005_01442_amd import _abi

    return _abi


def test_every_declared_symbol_is_exported(abi):
    names = _declared_functions()
    assert len(names) >= 18
    lib = ctypes.CDLL(LIB)
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(abi.PROTOTYPES), set(names) ^ set(abi.PROTOTYPES)
    nm = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (vr_\w+)", nm))
    assert set(names) <= exported


def test_abi_version(abi):
    assert abi.lib().vr_abi_version() == abi.VR_ABI_VERSION == 2


def test_struct_layout_matches_the_header(abi, tmp_path):
    """sizeof/offsetof from the C compiler against the ctypes mirror."""
    checks = {
        "vr_volume": ["data", "dtype", "nx", "nz"],
        "vr_camera": ["projection", "width", "eye", "forward", "fov_y", "ortho_h"],
        "vr_tf": ["table", "K", "v0", "v1"],
        "vr_params": ["step", "ert_threshold", "use_skip", "counters"],
        "vr_shading": ["ambient", "shininess", "light", "headlight", "grad_min"],
        "vr_serve_config": ["hbm_budget_bytes", "max_inflight", "max_batch_tiles", "device", "brick_pool_bytes"],
        "vr_request": ["volume_id", "K", "tf_table_host", "tf_v1", "cam", "step", "use_skip"],
        "vr_serve_stats": ["submitted", "tiles", "p50_ms", "p99_ms", "busy_s", "samples", "samples_per_s",
                           "queued_max", "queued_mean", "resident_bytes"],
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "vr.h"', "int main(void){"]
    for s, fields in checks.items():
        lines.append(f'printf("{s} %zu\\n", sizeof({s}));')
        for f in fields:
            lines.append(f'printf("{s}.{f} %zu\\n", offsetof({s}, {f}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = dict(line.split() for line in out if line.strip())
    for s, fields in checks.items():
        cls = getattr(abi, s)
        assert int(got[s]) == ctypes.sizeof(cls), s
        for f in fields:
            assert int(got[f"{s}.{f}"]) == getattr(cls, f).offset, (s, f)


def test_validation_without_device(abi):
    L = abi.lib()
    vol = abi.vr_volume(None, abi.VR_I16, 0, 8, 8, 8)
    cam = abi.vr_camera()
    tf = abi.vr_tf(None, 256, 0.0, 1.0)
    p = abi.vr_params(0.5, 0.0, 0, 0, None)
    rc = L.vr_render(ctypes.byref(vol), None, ctypes.byref(cam), 1, ctypes.byref(tf), ctypes.byref(p), None, None)
    assert rc == 1 and b"volume data is NULL" in L.vr_last_error()
    vol.data = 4096  # a non-null address that is never dereferenced: validation stops first
    rc = L.vr_render(ctypes.byref(vol), None, ctypes.byref(cam), 1, ctypes.byref(tf), ctypes.byref(p), None, None)
    assert rc == 1 and b"TF table is NULL" in L.vr_last_error()
    tf.table = 4096
    tf.K = 1
    rc = L.vr_render(ctypes.byref(vol), None, ctypes.byref(cam), 1, ctypes.byref(tf), ctypes.byref(p), None, None)
    assert rc == 1 and b"K=1" in L.vr_last_error()
    tf.K = 256
    p.step = -1.0
    rc = L.vr_render(ctypes.byref(vol), None, ctypes.byref(cam), 1, ctypes.byref(tf), ctypes.byref(p), None, None)
    assert rc == 1 and b"step" in L.vr_last_error()
    p.step = 0.5
    rc = L.vr_render(ctypes.byref(vol), None, ctypes.byref(cam), 1, ctypes.byref(tf), ctypes.byref(p), None, None)
    assert rc == 1 and b"image size" in L.vr_last_error()
    cam.width = cam.height = 8
    cam.projection = 1
    cam.forward[2] = 1.0
    cam.fov_y = 4.0
    rc = L.vr_render(ctypes.byref(vol), None, ctypes.byref(cam), 1, ctypes.byref(tf), ctypes.byref(p), None, None)
    assert rc == 1 and b"fov_y" in L.vr_last_error()
    cam.fov_y = 1.0
    p.use_skip = 1
    rc = L.vr_render(ctypes.byref(vol), None, ctypes.byref(cam), 1, ctypes.byref(tf), ctypes.byref(p), None, None)
    assert rc == 1 and b"use_skip needs blocks" in L.vr_last_error()
    p.use_skip = 0
    rc = L.vr_render(ctypes.byref(vol), None, ctypes.byref(cam), 0, ctypes.byref(tf), ctypes.byref(p), None, None)
    assert rc == 1 and b"at least one camera" in L.vr_last_error()
    p.use_skip = 1
    vol.nx = 1 << 21
    rc = L.vr_render(ctypes.byref(vol), None, ctypes.byref(cam), 1, ctypes.byref(tf), ctypes.byref(p), None, None)
    assert rc == 2  # VR_E_UNSUPPORTED: over the per-volume size limit
    out = ctypes.c_void_p()
    rc = L.vr_build_blocks(ctypes.byref(abi.vr_volume(4096, abi.VR_I16, 0, 8, 8, 8)), 2, None, ctypes.byref(out))
    assert rc == 1 and b"block edge" in L.vr_last_error()
    rc = L.vr_build_blocks(ctypes.byref(abi.vr_volume(4096, abi.VR_I16, 0, 8, 8, 8)), 12, None, ctypes.byref(out))
    assert rc == 1 and b"power of two" in L.vr_last_error()


def test_timeline_only_in_the_diagnostics_build(abi):
    """The product library keeps no per-wavefront timeline."""
    L = abi.lib()
    n = ctypes.c_uint64(7)
    buf = (ctypes.c_uint64 * 8)()
    assert L.vr_timeline_read(0, ctypes.cast(buf, ctypes.c_void_p), 2, ctypes.byref(n)) == 2  # VR_E_UNSUPPORTED
    assert b"VR_TIMELINE" in L.vr_last_error()
    assert n.value == 7


def test_serve_config_validation_without_device(abi):
    L = abi.lib()
    out = ctypes.c_void_p()
    cfg = abi.vr_serve_config(0, 4, 0, 0, 0)
    assert L.vr_serve_create(ctypes.byref(cfg), ctypes.byref(out)) == 1
    cfg = abi.vr_serve_config(1 << 20, 0, 0, 0, 0)
    assert L.vr_serve_create(ctypes.byref(cfg), ctypes.byref(out)) == 1
    assert b"max_inflight" in L.vr_last_error()


def test_shading_validation_without_device(abi):
    L = abi.lib()
    vol = abi.vr_volume(4096, abi.VR_I16, 0, 8, 8, 8)
    cam = abi.vr_camera()
    cam.width = cam.height = 8
    cam.projection = 1
    cam.forward[2] = 1.0
    cam.right[0] = 1.0
    cam.up[1] = 1.0
    cam.fov_y = 1.0
    tf = abi.vr_tf(4096, 256, 0.0, 1.0)
    p = abi.vr_params(0.5, 0.0, 0, 0, None)
    args = lambda sh: (ctypes.byref(vol), None, ctypes.byref(cam), 1, ctypes.byref(tf), ctypes.byref(p),  # noqa: E731
                       sh, None, None)
    assert L.vr_render_shaded(*args(None)) == 1 and b"shading is NULL" in L.vr_last_error()
    sh = abi.vr_shading(0.3, 0.7, 0.3, 16.0, (ctypes.c_float * 3)(0.0, 0.0, 0.0), 0, 1.0, 0)
    assert L.vr_render_shaded(*args(ctypes.byref(sh))) == 1 and b"zero length" in L.vr_last_error()
    sh.headlight = 1
    sh.shininess = 0.5
    assert L.vr_render_shaded(*args(ctypes.byref(sh))) == 1 and b"shininess" in L.vr_last_error()
    sh.shininess = 16.0
    sh.grad_min = 0.0
    assert L.vr_render_shaded(*args(ctypes.byref(sh))) == 1 and b"grad_min" in L.vr_last_error()
    sh.grad_min = 1.0
    sh.specular = float("nan")
    assert L.vr_render_shaded(*args(ctypes.byref(sh))) == 1 and b"specular" in L.vr_last_error()
    sh.specular = 0.3
    # a valid shading reaches the output check (nothing is enqueued)
    assert L.vr_render_shaded(*args(ctypes.byref(sh))) == 1 and b"out_rgba is NULL" in L.vr_last_error()
