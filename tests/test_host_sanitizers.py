"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Builds a copy of libts.so whose host code (every .cpp source: setup
eigensolvers, SEM and Hermite assembly, the C ABI and the task / serving
logic) is compiled with -fsanitize=address,undefined, and a sanitized copy of
the oracle's C core, then reruns the host-side test files against them in a
child Python with the sanitizer runtime preloaded.  Any invalid access, leak
of a freed block, misaligned or overflowing arithmetic aborts the child.
A planted heap overflow in a throwaway library shows that the harness
catches such errors.  Device code is not instrumented (GPU sanitizers are
not used), and entry points that need a GPU are not exercised here.
"""
import glob
import os
import subprocess
import sys

import pytest

import oracle
from paper_2605_20491_amd import build as libbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

# host entry points of the library (setup eigensolvers, SEM / Hermite axes,
# quadrature, BF16 rounding) and the oracle's axis, dense and apply kernels on
# small grids (the oracle runs serially here, so its large pins stay out)
HOST_TESTS = ["tests/test_lib_host.py", "tests/test_lib_bf16_round.py", "tests/test_oracle_axis.py",
              "tests/test_oracle_apply.py::test_inverse_matches_dense_lu",
              "tests/test_oracle_apply.py::test_exp_matches_dense_expm"]


def _asan_runtime():
    libs = glob.glob(os.path.join(ROCM, "llvm", "lib", "clang", "*", "lib", "linux", "libclang_rt.asan-x86_64.so"))
    return libs[0] if libs else None


def _env(extra):
    env = dict(os.environ)
    env.update({"LD_PRELOAD": _asan_runtime(), "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1", "OMP_NUM_THREADS": "4"})
    env.update(extra)
    return env


@pytest.mark.skipif(_asan_runtime() is None, reason="ROCm's clang sanitizer runtime is not installed")
def test_host_code_under_address_and_ub_sanitizers(tmp_path):
    if not os.path.exists(os.path.join(ROOT, "paper_2605_20491_amd", "_build", "ts_api.o")):
        libbuild.build()
    lib = libbuild.build_sanitized(str(tmp_path))
    orc = oracle.build_sanitized(str(tmp_path / "_oracle.so"))
    clang = os.path.join(ROCM, "llvm", "bin", "clang")

    # the harness catches a planted heap overflow
    canary = tmp_path / "canary.c"
    canary.write_text("#include <stdlib.h>\nint poke(int n) { int* a = malloc(4 * n); a[n] = 1; "
                      "int r = a[0]; free(a); return r; }\n")
    subprocess.check_call([clang, "-O1", "-g", "-fsanitize=address", "-fPIC", "-shared", "-o",
                           str(tmp_path / "canary.so"), str(canary)])
    r = subprocess.run([sys.executable, "-c", "import ctypes; ctypes.CDLL(%r).poke(8)" % str(tmp_path / "canary.so")],
                       env=_env({}), capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr

    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider"]
                       + HOST_TESTS, cwd=ROOT, env=_env({"TS_LIBRARY": lib, "ORACLE_LIBRARY": orc}),
                       capture_output=True, text=True, timeout=1500)
    out = r.stdout + r.stderr
    print(out[-3000:])
    assert r.returncode == 0, out[-3000:]
    assert "AddressSanitizer" not in out and "runtime error:" not in out
