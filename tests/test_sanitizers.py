"""Host sanitizer runs (CPU only): the oracle, and the library's host code on
its validation and error paths, built with AddressSanitizer and
UndefinedBehaviorSanitizer and driven by the C programs in tests/sanitize/.

The library's kernels are not instrumented: only the host translation unit
(the C-ABI, argument checks, staging, workspace and graph bookkeeping) carries
the sanitizers; it is linked with the kernels' ordinary objects.  A run passes
when the driver's own expectations hold and no sanitizer report is raised
(any report aborts the program: recovery is off).  Device paths are covered by
the GPU tests; with a GPU present these runs are skipped, since the sanitizer
runtime and the HIP runtime's address-space reservations are not meant to
share a process.
"""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
PKG = os.path.join(ROOT, "paper_1801_01072_amd")
ROCM = "/opt/rocm"
CLANG = os.path.join(ROCM, "llvm", "bin", "clang")
CLANGXX = os.path.join(ROCM, "llvm", "bin", "clang++")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]
SANITIZE = ["-fsanitize=address,undefined"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")

pytestmark = pytest.mark.skipif(os.path.exists("/dev/kfd"),
                                reason="host-only sanitizer runs; a GPU is present")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r


def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not found")
    exe = str(tmp_path / "oracle_san")
    _run(["gcc", "-std=gnu11", *FLAGS, *SANITIZE, "-static-libasan", "-static-libubsan",
          os.path.join(SAN, "oracle_driver.c"), "-lm", "-o", exe])
    r = _run([exe], env=ENV, timeout=300)
    assert "oracle sanitizer run: ok" in r.stdout


def test_library_host_code_under_address_and_undefined_sanitizers(tmp_path):
    objs = sorted(o for o in glob.glob(os.path.join(PKG, "_build", "*.o"))
                  if not os.path.basename(o).startswith("engine.cpp"))
    if not objs or not os.path.exists(HIPCC) or not os.path.exists(CLANGXX):
        pytest.skip("library objects or the ROCm toolchain are missing (run the build first)")
    inc = [f"-I{os.path.join(ROOT, 'include')}", f"-I{os.path.join(PKG, 'csrc')}"]
    eng = str(tmp_path / "engine_san.o")
    # host pass only: each sanitizer flag is scoped to the host compilation
    _run([HIPCC, "-x", "hip", "--offload-arch=gfx950", "-std=c++17", "-fPIC", *FLAGS,
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *inc,
          "-c", os.path.join(PKG, "csrc", "engine.cpp"), "-o", eng])
    drv = str(tmp_path / "abi_driver.o")
    _run([CLANG, "-std=gnu11", *FLAGS, *SANITIZE, *inc, "-c", os.path.join(SAN, "abi_driver.c"),
          "-o", drv])
    exe = str(tmp_path / "abi_san")
    _run([CLANGXX, *SANITIZE, drv, eng, *objs, f"-L{ROCM}/lib", "-lamdhip64",
          f"-Wl,-rpath,{ROCM}/lib", "-o", exe])
    r = _run([exe], env=ENV, timeout=300)
    assert "abi sanitizer run: ok" in r.stdout
