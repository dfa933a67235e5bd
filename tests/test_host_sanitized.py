"""The host planner under AddressSanitizer and UndefinedBehaviorSanitizer.

Builds a second copy of the library whose host sources (the exact integer
planner, the pyramid driver, the batch scheduler, the C ABI) are compiled
with g++ -fsanitize=address,undefined and linked with the unmodified gfx950
objects of the regular build, then runs the CPU ctypes tests of
test_host_planner.py and test_host_tune_cache.py (the tuning cache's JSON
reader on good and malformed files) against it in a child process (the library is selected
with LFFT_LIBRARY).  Any sanitizer report aborts the child and fails the test.
No GPU is used: every plan in those tests is host-only.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1107_5415_amd", "csrc")
OBJ = os.path.join(ROOT, "_build")
OUT = os.path.join(ROOT, "_build", "sanitized")
HOST_SOURCES = ["intmat.cpp", "plan.cpp", "capi.cpp", "batch.cpp", "ktrace.cpp", "wave.cpp",
                "tune_cache.cpp", "planlog.cpp"]
FLAGS = ["-O1", "-g", "-std=c++17", "-fPIC", "-fsanitize=address,undefined",
         "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined", "-D__HIP_PLATFORM_AMD__",
         "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
         "-Wno-unknown-pragmas"]


def _device_objects():
    if not os.path.isdir(OBJ):
        return []
    return sorted(os.path.join(OBJ, f) for f in os.listdir(OBJ) if f.endswith(".hip.o"))


def _build():
    os.makedirs(OUT, exist_ok=True)

    def cc(src):
        obj = os.path.join(OUT, src + ".o")
        r = subprocess.run(["g++"] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj],
                           capture_output=True, text=True)
        if r.returncode:
            raise RuntimeError(r.stderr)
        return obj
    with cf.ThreadPoolExecutor(max_workers=6) as ex:
        objs = list(ex.map(cc, HOST_SOURCES))
    lib = os.path.join(OUT, "liblfft_sanitized.so")
    r = subprocess.run(["g++", "-shared", "-fsanitize=address,undefined", "-o", lib] + objs +
                       _device_objects() + ["-L/opt/rocm/lib", "-lamdhip64",
                                            "-Wl,-rpath,/opt/rocm/lib"],
                       capture_output=True, text=True)
    if r.returncode:
        raise RuntimeError(r.stderr)
    return lib


def _runtime(name):
    p = subprocess.run(["gcc", "-print-file-name=" + name], capture_output=True, text=True).stdout.strip()
    return p if os.path.isabs(p) and os.path.exists(p) else None


@pytest.mark.skipif(not _device_objects(), reason="regular build objects missing (run build())")
def test_host_planner_sanitized():
    asan, stdcxx = _runtime("libasan.so"), _runtime("libstdc++.so")
    if not asan or not stdcxx:
        pytest.skip("sanitizer runtime not found")
    lib = _build()
    env = dict(os.environ)
    env.update(LFFT_LIBRARY=lib,
               # the sanitizer runtime first; libstdc++ so that its exception
               # interceptors resolve in a Python host process
               LD_PRELOAD=asan + " " + stdcxx,
               ASAN_OPTIONS="detect_leaks=0:protect_shadow_gap=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_host_planner.py"),
                        os.path.join(ROOT, "tests", "test_host_tune_cache.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
