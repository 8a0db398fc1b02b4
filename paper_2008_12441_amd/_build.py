"""Build libhmat.so in-tree for gfx950 (hipcc for the kernels, g++ for the host side)."""
from __future__ import annotations

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "lib", "libhmat.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", f"-I{INCLUDE}", f"-I{CSRC}"]
HOST_SOURCES = ["hmat_host.cpp", "hmat_batch_host.cpp", "hmat_structure.cpp", "hmat_h2_host.cpp"]
HIP_SOURCES = ["hmat_kernels.hip", "hmat_mr_kernels.hip", "hmat_batch.hip", "hmat_compress.hip", "hmat_h2.hip"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-Wextra", "-D__HIP_PLATFORM_AMD__",
              f"-I{ROCM}/include", f"-I{INCLUDE}", f"-I{CSRC}"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = False) -> str:
    """Compile every source of the library and link it; always rebuilds."""
    os.makedirs(BUILD, exist_ok=True)
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    jobs = []
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        jobs.append((["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj], obj))
    for src in HIP_SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        jobs.append(([os.path.join(ROCM, "bin", "hipcc"), *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj], obj))
    # the sources compile independently; a few at a time bounds the memory the compilers take
    workers = max(1, min(len(jobs), int(os.environ.get("HMAT_BUILD_JOBS", "4"))))
    with ThreadPoolExecutor(max_workers=workers) as pool:
        list(pool.map(lambda j: _run(j[0], verbose), jobs))
    objs = [obj for _, obj in jobs]
    tmp = LIB + ".tmp"
    _run([os.path.join(ROCM, "bin", "hipcc"), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp,
          "-lpthread"], verbose)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
