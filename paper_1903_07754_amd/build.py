"""Build libwedge.so for gfx950 in-tree.

Host C++ (api.cpp, layout.cpp) is compiled with g++, the HIP kernels with
hipcc for gfx950, and the objects are linked by hipcc into a shared library
next to this file. Packed FP32 instructions are disabled for device code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libwedge.so")
LIB_DEBUG = os.path.join(HERE, "libwedge_debug.so")
LIB_ASAN = os.path.join(HERE, "libwedge_asan.so")
SANITIZE = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
            "-fno-sanitize-recover=undefined"]
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
ARCH = "gfx950"

HIPCC_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Wno-unused-command-line-argument"]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", "-D__HIP_PLATFORM_AMD__",
              f"-I{ROCM}/include"]


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = False, debug_checks: bool = False) -> str:
    """Compile libwedge.so; debug_checks builds libwedge_debug.so instead, with the
    device checks of WEDGE_DEBUG_CHECKS compiled in (index, destination and
    in-edge checks in the pulls, the translation and the chunk lists; a failed
    check makes the run return WEDGE_ERR_HIP). Load it with WEDGE_LIB=<path>."""
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    obj_dir = os.path.join(HERE, "_build", "debug" if debug_checks else "")
    os.makedirs(obj_dir, exist_ok=True)
    extra = ["-DWEDGE_DEBUG_CHECKS"] if debug_checks else []
    lib = LIB_DEBUG if debug_checks else LIB
    objs = []
    for src in ("api.cpp", "layout.cpp", "model.cpp"):
        o = os.path.join(obj_dir, src + ".o")
        _run(["g++", *HOST_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", o], verbose)
        objs.append(o)
    for src in ("kernels.hip", "batch.hip", "mlp.hip", "noalloc.hip", "push.hip"):
        o = os.path.join(obj_dir, src + ".o")
        _run([hipcc, *HIPCC_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", o], verbose)
        objs.append(o)
    tmp = lib + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-lpthread",
          f"-L{ROCM}/lib", "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{ROCM}/lib"], verbose)
    os.replace(tmp, lib)
    return lib


def build_sanitized(verbose: bool = False) -> str:
    """libwedge_asan.so: the host C++ (argument checks, layout build, model
    files, tuner cache) under AddressSanitizer and UBSan, linked with the
    release build's device objects (build() first). For host-only tests:
    load it with WEDGE_LIB and the sanitizer runtimes preloaded."""
    hipcc = shutil.which("hipcc") or os.path.join(ROCM, "bin", "hipcc")
    rel = os.path.join(HERE, "_build")
    obj_dir = os.path.join(HERE, "_build", "asan")
    os.makedirs(obj_dir, exist_ok=True)
    objs = []
    for src in ("api.cpp", "layout.cpp", "model.cpp"):
        o = os.path.join(obj_dir, src + ".o")
        flags = [f for f in HOST_FLAGS if f != "-O2"]
        _run(["g++", *flags, *SANITIZE, "-c", os.path.join(CSRC, src), "-o", o], verbose)
        objs.append(o)
    for src in ("kernels.hip", "batch.hip", "mlp.hip", "noalloc.hip", "push.hip"):
        objs.append(os.path.join(rel, src + ".o"))
    tmp = LIB_ASAN + ".tmp"
    _run([hipcc, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-lpthread",
          f"-L{ROCM}/lib", "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{ROCM}/lib", "-lasan", "-lubsan"],
         verbose)
    os.replace(tmp, LIB_ASAN)
    return LIB_ASAN


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, debug_checks="--debug-checks" in sys.argv))
