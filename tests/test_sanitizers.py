"""Host code under the sanitizers (CPU only; the drivers are in
tests/sanitize/):
  * the C oracle, driven through every entry point on small seeded inputs and
    edge cases, under AddressSanitizer and UndefinedBehaviorSanitizer;
  * the library's host-side paths (argument validation of every C-ABI entry
    point, the host-only brick ordering), built with those two sanitizers on
    the host side of every HIP source;
  * the serving scheduler's threads (scheduler, out-of-core worker, clients,
    statistics and volume registration) under ThreadSanitizer, with a CPU
    stand-in for the device operations (vr::ServeOps)."""

import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2005_01442_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ENV = dict(os.environ, UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ... failed ({r.returncode}):\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-std=c11", "-O1", "-g", "-fopenmp", "-ffp-contract=off", "-fno-omit-frame-pointer",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-o", exe,
          os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(SAN, "oracle_driver.c"), "-lm"])
    r = _run([exe], env=dict(ENV, ASAN_OPTIONS="detect_leaks=1"))
    assert "oracle driver: ok" in r.stdout


def _build_library_with(driver, sanitizers, tmp_path):
    """Every library source plus `driver`, the sanitizers on the host side."""
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp")))
    srcs.append(os.path.join(SAN, driver))
    san = []
    for x in sanitizers:
        san += ["-Xarch_host", x]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-ffp-contract=off",
             "-munsafe-fp-atomics", "-fno-omit-frame-pointer", *san]

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        _run([HIPCC, *flags, "-c", src, "-o", obj])
        return obj

    with ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(tmp_path / (os.path.splitext(driver)[0] + ".exe"))
    _run([HIPCC, "--offload-arch=gfx950", *san, "-pthread", "-o", exe, *objs])
    return exe


HAVE_HIPCC = shutil.which(HIPCC) is not None or os.path.exists(HIPCC)


@pytest.mark.skipif(not HAVE_HIPCC, reason="hipcc not available")
def test_library_host_code_under_asan_and_ubsan(tmp_path):
    exe = _build_library_with("abi_driver.cpp", ["-fsanitize=address", "-fsanitize=undefined"], tmp_path)
    # the HIP runtime (not instrumented) keeps allocations until exit: no leak check
    r = _run([exe], env=dict(ENV, ASAN_OPTIONS="detect_leaks=0"))
    assert "abi driver: ok" in r.stdout


@pytest.mark.skipif(not HAVE_HIPCC, reason="hipcc not available")
def test_serving_threads_under_tsan_with_a_cpu_stand_in(tmp_path):
    exe = _build_library_with("serve_tsan_driver.cpp", ["-fsanitize=thread"], tmp_path)
    r = _run([exe], env=dict(ENV, TSAN_OPTIONS="halt_on_error=1:second_deadlock_stack=1"))
    assert "serve tsan driver: ok" in r.stdout and "WARNING: ThreadSanitizer" not in r.stderr
