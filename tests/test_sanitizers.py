"""Host-side AddressSanitizer / UndefinedBehaviorSanitizer runs (no GPU).

- The oracle's C code, compiled with gcc under both sanitizers into a driver
  (tests/sanitize/oracle_driver.c) that calls every exported routine on small
  meshes of every boundary-condition kind and degree.
- The library's host code (reference element, argument checks of every entry
  point), built with hipcc with the sanitizers on the host side only, driven
  by tests/sanitize/capi_driver.cpp.

A report from either sanitizer (out-of-bounds access, use after free, leak,
undefined arithmetic) ends the driver with a non-zero status."""
import hashlib
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2504_00998_amd", "csrc")
LIB_SOURCES = ["fe_api.cpp", "fe_refelem.cpp", "fe_dense.cpp", "fe_adjoint.cpp", "fe_kernels.hip",
               "fe_nonlocal.hip", "fe_density.hip", "fe_poisson.hip"]
HIPCC = "/opt/rocm/bin/hipcc"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{cmd[0]} failed ({r.returncode}):\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_c_is_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-std=c11", "-D_DEFAULT_SOURCE", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-o", exe, os.path.join(HERE, "oracle_driver.c"), "-lm"])
    r = _run([exe], env=ENV, timeout=600)
    assert "done" in r.stdout


def _asan_library():
    """Host-sanitized build of the library in a temporary folder, reused while
    the sources are unchanged (the device code is built as usual)."""
    h = hashlib.sha256()
    for s in LIB_SOURCES + ["fe_internal.h"]:
        h.update(open(os.path.join(CSRC, s), "rb").read())
    h.update(open(os.path.join(ROOT, "include", "fe.h"), "rb").read())
    d = os.path.join(tempfile.gettempdir(), "fe_asan_" + h.hexdigest()[:16])
    lib = os.path.join(d, "libfe_asan.so")
    if not os.path.exists(lib):
        os.makedirs(d, exist_ok=True)
        tmp = lib + ".tmp"
        _run([HIPCC, "-std=c++17", "-fPIC", "-shared", "--offload-arch=gfx950", "-O1", "-g", "-fno-omit-frame-pointer",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
              "-I" + os.path.join(ROOT, "include"), "-o", tmp] + [os.path.join(CSRC, s) for s in LIB_SOURCES]
             + ["-L/opt/rocm/lib", "-lrocblas", "-lrocsolver", "-Wl,-rpath,/opt/rocm/lib"], timeout=1200)
        os.replace(tmp, lib)
    return d


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="needs hipcc")
def test_capi_host_paths_are_clean_under_asan_and_ubsan(tmp_path):
    d = _asan_library()
    exe = str(tmp_path / "capi_driver")
    _run([HIPCC, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-I" + os.path.join(ROOT, "include"), "-o", exe, os.path.join(HERE, "capi_driver.cpp"),
          "-L" + d, "-lfe_asan", "-Wl,-rpath," + d, "-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib"],
         timeout=600)
    r = _run([exe], env=ENV, timeout=600)
    assert "done" in r.stdout
