"""Build ``libpwf.so`` (HIP, gfx950) in-tree with hipcc.

Each translation unit is compiled in parallel into ``_build/`` and linked
into ``paper_2503_20146_amd/libpwf.so``.  Run ``python -m
paper_2503_20146_amd.build`` or call :func:`build`.
"""

from __future__ import annotations

import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libpwf.so")

ARCH = "gfx950"
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    # no packed FP32 instructions in generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def _hipcc() -> str:
    for cand in (shutil.which("hipcc"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found: the HIP toolchain is required to build libpwf")


def sources() -> list[str]:
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src)[:-4] + ".o")
    cmd = [_hipcc(), *FLAGS, "-c", src, "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stdout}\n{res.stderr}")
    return obj


def build(jobs: int | None = None, verbose: bool = True) -> str:
    """Compile every HIP source and link libpwf.so; returns the library path."""
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), max(1, min(os.cpu_count() or 1, 16)))
    if verbose:
        print(f"[build] hipcc {ARCH}: {len(srcs)} sources, {jobs} jobs", flush=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    if verbose:
        print(f"[build] wrote {LIB}", flush=True)
    return LIB


C_CONSUMER = os.path.join(ROOT, "tests", "c_consumer", "pwf_c_solve")


def build_c_consumer(verbose: bool = True) -> str | None:
    """Compile the tests' C99 consumer of the library (tests/c_consumer/pwf_c_solve.c: a
    plain C program that runs pwf_solve with the HIP runtime for memory and a stream) with
    gcc against include/pwf.h and libpwf.so; returns its path, or None without gcc."""
    gcc = shutil.which("gcc")
    if gcc is None:
        if verbose:
            print("[build] gcc not found: the C consumer of the tests is not built", flush=True)
        return None
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cmd = [gcc, "-std=c99", "-O2", "-Wall", "-Wextra", "-pedantic", "-Werror", "-D__HIP_PLATFORM_AMD__",
           "-isystem", os.path.join(rocm, "include"), "-I", os.path.join(ROOT, "include"), C_CONSUMER + ".c",
           "-o", C_CONSUMER, "-L", os.path.join(rocm, "lib"), "-lamdhip64", "-L", PKG, "-lpwf",
           f"-Wl,-rpath,{PKG}", f"-Wl,-rpath,{os.path.join(rocm, 'lib')}"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"C consumer build failed:\n{res.stdout}\n{res.stderr}")
    if verbose:
        print(f"[build] wrote {C_CONSUMER}", flush=True)
    return C_CONSUMER


if __name__ == "__main__":
    build(int(sys.argv[1]) if len(sys.argv) > 1 else None)
