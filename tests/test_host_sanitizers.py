"""Host code of libbf under AddressSanitizer and UndefinedBehaviorSanitizer (CPU).

The library is rebuilt with the sanitizers on its host code only (every
`-fsanitize=` follows `-Xarch_host`; the device code is built as usual), and
the host-side test modules -- the ABI checks (validation of every
description field, plan-free entry points, thread-local errors, the demod and
envelope validators) and the binding's argument checks -- run against it in a
child process with the sanitizer runtime preloaded.  Any sanitizer report
aborts the child, so the run fails.  Without a GPU the device entry points
return BF_ERR_NO_DEVICE after validation, so this covers the validation,
table-building and error paths that run before any device call.
"""
import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2512_11086_amd", "csrc")
SOURCES = ["bf_api", "bf_batch", "bf_decode", "bf_das", "bf_das_lds", "bf_das_adj", "bf_adjoint",
           "bf_demod", "bf_env"]
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]


def _runtime():
    hits = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_host_code_under_asan_and_ubsan(tmp_path):
    import torch
    if torch.cuda.is_available():
        pytest.skip("host-only check; a GPU is present")
    rt = _runtime()
    if rt is None:
        pytest.skip("no AddressSanitizer runtime in this ROCm image")
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    base = [hipcc, "-O1", "-g", "-fPIC", "-std=c++17", "--offload-arch=gfx950",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Xarch_host", "-fno-omit-frame-pointer", *SAN,
            "-I", os.path.join(ROOT, "include"), "-I", CSRC]

    def compile_one(name):
        obj = str(tmp_path / f"{name}.o")
        r = subprocess.run(base + ["-c", os.path.join(CSRC, name + ".hip"), "-o", obj],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        return obj

    with ThreadPoolExecutor(max_workers=8) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    lib = str(tmp_path / "libbf_san.so")
    r = subprocess.run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", *SAN, "-shared-libsan",
                        "-o", lib, *objs], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, BF_LIBRARY=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x",
                        os.path.join(ROOT, "tests", "test_abi.py"),
                        os.path.join(ROOT, "tests", "test_binding_checks.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
