"""Build the gfx950 HIP library ``libvr.so`` in-tree with hipcc.

Every source under ``csrc/`` is compiled for gfx950 only, with packed-FP32
instructions disabled, and linked into one shared library exporting the C ABI
of ``include/vr.h``.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libvr.so")
BUILD_DIR = os.path.join(ROOT, "_build", "vr")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
COMMON = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-fPIC",
    "-std=c++17",
    "-I", INCLUDE,
    "-I", CSRC,
    "-Wall",
    "-Wno-unused-result",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no implicit FMA contraction: every fused multiply-add is written out, so
    # kernels that share device functions (the whole-image render, the
    # serving kernel, the out-of-core pass) compute bit-identical samples
    "-ffp-contract=off",
    "-munsafe-fp-atomics",
]


def sources():
    return sorted(
        os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip") or f.endswith(".cpp")
    )


def _compile(src, extra=(), build_dir=BUILD_DIR):
    obj = os.path.join(build_dir, os.path.basename(src) + ".o")
    cmd = [HIPCC, *COMMON, *extra, "-c", src, "-o", obj]
    if src.endswith(".cpp"):
        cmd += ["-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    errs = "\n".join(
        ln for ln in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in ln
    )
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{errs}")
    return obj, errs


def build(verbose: bool = False, extra=(), out: str = LIB) -> str:
    """Compile and link; ``extra`` adds compiler flags, ``out`` names the
    library (tuning variants are built beside the default one)."""
    build_dir = BUILD_DIR if out == LIB else os.path.join(BUILD_DIR, os.path.basename(out))
    os.makedirs(build_dir, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        results = list(ex.map(lambda src: _compile(src, tuple(extra), build_dir), srcs))
    for _, errs in results:
        if verbose and errs.strip():
            print(errs, file=sys.stderr)
    objs = [o for o, _ in results]
    tmp = out + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs]
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
