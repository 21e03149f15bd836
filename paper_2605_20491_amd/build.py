"""Build libts.so (HIP kernels for gfx950 + the C ABI) in-tree with hipcc.

Every source is compiled with hipcc for --offload-arch=gfx950 and linked into
paper_2605_20491_amd/libts.so.  Objects go to paper_2605_20491_amd/_build/.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libts.so")

SOURCES = ["eig_tridiag.cpp", "sem_setup.cpp", "ts_api.cpp", "solvers.cpp", "modeprod.hip", "modeprod_bf16.hip", "modeprod_small.hip", "small_plan.cpp", "split.cpp", "serve.cpp", "vec.hip", "gpe.cpp", "gpe_kernels.hip", "multilevel.hip", "hermite.cpp", "noalloc.cpp"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    # keep packed FP32 instructions out of the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-I", CSRC,
    "-Wno-unused-result",
]


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, src.rsplit(".", 1)[0] + ".o")
    path = os.path.join(CSRC, src)
    cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", path, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, r.stdout, r.stderr))
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(_compile, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (r.stdout, r.stderr))
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def build_sanitized(outdir: str, verbose: bool = False) -> str:
    """A copy of libts.so whose host code (every .cpp source) is compiled with
    the address and undefined-behaviour sanitizers; device code and the .hip
    sources are the regular objects (GPU sanitizers are not used).  Needs the
    regular objects of build() in _build/."""
    os.makedirs(outdir, exist_ok=True)
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer", "-g"]

    def one(src):
        if not src.endswith(".cpp"):
            return os.path.join(BUILD, src.rsplit(".", 1)[0] + ".o")
        obj = os.path.join(outdir, src.rsplit(".", 1)[0] + ".o")
        cmd = [HIPCC] + FLAGS + san + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc (sanitized) failed for %s:\n%s\n%s" % (src, r.stdout, r.stderr))
        return obj

    with cf.ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(one, SOURCES))
    lib = os.path.join(outdir, "libts.so")
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-shared-libsan", "-o", lib] + objs + ["-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("sanitized link failed:\n%s\n%s" % (r.stdout, r.stderr))
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
