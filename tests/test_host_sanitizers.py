"""The host side of the library (argument validation, workspace sizing, plan bookkeeping in
api.cpp) run under AddressSanitizer and UndefinedBehaviorSanitizer: api.cpp is rebuilt with
both on its host pass, linked with the ordinary device objects, and the CPU-only ABI,
binding and checkpoint tests run against that build in a child process (SOP_LIBRARY points
the binding at it). Any sanitizer report fails the test. No device code is instrumented and
no GPU is touched."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from paper_2510_07729_amd import build as B   # noqa: E402

# sanitizers on the host pass only
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def asan_runtime():
    hits = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    return hits[0] if hits else None


def test_host_library_under_asan_and_ubsan(tmp_path):
    rt = asan_runtime()
    if rt is None or not os.path.exists(B.hipcc()):
        pytest.skip("the compiler's AddressSanitizer runtime is not installed")
    os.makedirs(B.BUILD_DIR, exist_ok=True)
    objs = []
    for src in B.SOURCES:
        if src.endswith(".cpp"):
            continue
        obj = os.path.join(B.BUILD_DIR, os.path.splitext(src)[0] + ".o")
        if not os.path.exists(obj):
            obj = B._compile(src)
        objs.append(obj)
    api_o = str(tmp_path / "api_san.o")
    lib = str(tmp_path / "libsop_san.so")
    cc = [B.hipcc(), "-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={B.ARCH}",
          *HOST_SAN, "-x", "hip", "-c", os.path.join(B.CSRC, "api.cpp"), "-o", api_o]
    r = subprocess.run(cc, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    ld = [B.hipcc(), f"--offload-arch={B.ARCH}", "-shared", "-fPIC", *HOST_SAN,
          "-shared-libsan", api_o, *objs, "-o", lib]
    r = subprocess.run(ld, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ)
    env.update(SOP_LIBRARY=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    tests = [os.path.join(ROOT, "tests", t) for t in
             ("test_abi.py", "test_binding_checks.py", "test_checkpoint.py")]
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", *tests], capture_output=True, text=True, env=env,
                       cwd=str(tmp_path), timeout=600)
    out = r.stdout + r.stderr
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
