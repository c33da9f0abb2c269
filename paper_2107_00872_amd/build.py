"""Build libqs3.so (HIP for gfx950) in-tree.

hipcc compiles every source for gfx950 only; packed FP32 instructions are
disabled (-packed-fp32-ops) throughout.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
ROOT = os.path.dirname(PKG)
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libqs3.so")
SOURCES = ["capi.cpp", "hv.hip", "krylov.hip", "obs.hip", "server.cpp", "full.hip", "pg.hip", "noalloc.hip"]
# H.v / structure kernels: one translation unit per N_down
INST = [("hv_inst.hip", k) for k in range(0, 9)]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-x", "hip", "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-result", "-I", os.path.join(ROOT, "include")]


# the host-code sanitizer build: AddressSanitizer and UndefinedBehaviorSanitizer
# on the host side of every translation unit only (device code is unchanged);
# every sanitizer option is scoped to the host pass
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
CLANGXX = os.environ.get("QS3_CLANGXX", "/opt/rocm/llvm/bin/clang++")
HOST_CHECK = os.path.join(PKG, "qs3_host_check")


def _compile(item, build_dir: str = BUILD, extra_flags=()) -> str:
    src, k = item if isinstance(item, tuple) else (item, None)
    extra = [] if k is None else [f"-DQS3_INST_K={k}"]
    out = os.path.join(build_dir, src + ("" if k is None else f".k{k}") + ".o")
    cmd = [HIPCC, *FLAGS, *extra, *extra_flags, "-c", os.path.join(CSRC, src), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return out


def build(jobs: int = 8) -> str:
    os.makedirs(BUILD, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(_compile, INST + SOURCES))
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp, "-lpthread", "-lrocsolver", "-lrocblas"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB)
    return LIB


def build_host_check(jobs: int = 8) -> str:
    """The executable tests/host_abi_check.cpp linked against every library
    source built with the host-code sanitizers: it drives the C-ABI's host
    code (validation, structure builds, solver control, the serving
    scheduler) on a GPU with AddressSanitizer and UBSan watching."""
    bdir = os.path.join(BUILD, "host_san")
    os.makedirs(bdir, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda it: _compile(it, bdir, HOST_SAN), INST + SOURCES))
    drv = os.path.join(bdir, "host_abi_check.o")
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
    cmd = [CLANGXX, "-O1", "-g", "-std=c++17", *san, "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include",
           "-I", os.path.join(ROOT, "include"), "-c", os.path.join(ROOT, "tests", "host_abi_check.cpp"), "-o", drv]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    tmp = HOST_CHECK + ".tmp"
    cmd = [CLANGXX, *san, drv, *objs, "-o", tmp, "-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib",
           "-lamdhip64", "-lrocsolver", "-lrocblas", "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, HOST_CHECK)
    return HOST_CHECK


if __name__ == "__main__":
    print(build(int(sys.argv[1]) if len(sys.argv) > 1 else 8))
