"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: host.cpp and api.cpp
(validation, layout, step tables, splines, the C ABI's argument and error handling) are
rebuilt with both sanitizers on their host side, linked with the library's device objects
into a separate libcola, and the CPU tests of the C ABI run against it in a child process
with the sanitizer runtime preloaded.  Any report fails the run (halt_on_error).  No GPU
is used: these tests make no HIP calls beyond symbol loading."""

import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1703_00879_amd")
BUILD = os.path.join(PKG, "_build")
HIPCC = "/opt/rocm/bin/hipcc"
CLANG = "/opt/rocm/llvm/bin/clang++"


def _runtime():
    libs = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return libs[-1] if libs else None


@pytest.fixture(scope="module")
def sanitized_lib(tmp_path_factory):
    dev = [os.path.join(BUILD, f + ".o") for f in ("fft.hip", "pm.hip", "ic.hip", "noalloc.hip")]
    if not all(os.path.exists(f) for f in dev) or not os.path.exists(HIPCC) or not _runtime():
        pytest.skip("library objects or sanitizer runtime not available (run the build first)")
    d = tmp_path_factory.mktemp("asan")
    fl = ["-std=c++17", "-O1", "-g", "-fPIC", "--offload-arch=gfx950", "-fno-omit-frame-pointer",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-I", os.path.join(ROOT, "include"), "-I", os.path.join(PKG, "csrc"),
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    objs = []
    for src in ("host.cpp", "api.cpp"):
        o = str(d / (src + ".o"))
        subprocess.run([HIPCC] + fl + ["-c", os.path.join(PKG, "csrc", src), "-o", o], check=True,
                       capture_output=True)
        objs.append(o)
    lib = str(d / "libcola_sanitized.so")
    subprocess.run([CLANG, "-shared", "-fPIC", "-shared-libasan", "-fsanitize=address,undefined",
                    "-o", lib] + objs + dev + ["-L/opt/rocm/lib", "-lamdhip64",
                                               "-Wl,-rpath,/opt/rocm/lib"],
                   check=True, capture_output=True)
    return lib


def test_library_is_instrumented(sanitized_lib):
    syms = subprocess.run(["nm", "-D", sanitized_lib], capture_output=True, text=True).stdout
    assert "__asan_report_load" in syms and "__ubsan_handle_" in syms


def test_cpu_abi_tests_pass_under_sanitizers(sanitized_lib):
    env = dict(os.environ, COLA_LIBRARY=sanitized_lib, LD_PRELOAD=_runtime(),
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    tests = [os.path.join(ROOT, "tests", t) for t in
             ("test_abi.py", "test_tiles.py", "test_step_times.py", "test_bench_tools.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m",
                        "not gpu"] + tests, cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    out = r.stdout + r.stderr
    assert "ERROR: AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
