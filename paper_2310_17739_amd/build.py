"""Build the HIP library ``libqsim.so`` in-tree for gfx950.

Host sources are compiled by amdclang++ (no device code), the kernels by
hipcc for gfx950, and everything is linked into one shared library next to
this file.  Packed FP32 instructions are disabled in device code.
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
LIB = os.path.join(HERE, "libqsim.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")

HOST_SOURCES = ["gates.cpp", "fuse.cpp", "plan.cpp", "regplan.cpp", "qasm.cpp", "abi.cpp", "batch.cpp", "serve.cpp"]
DEVICE_SOURCES = ["kernels.hip"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          f"-I{os.path.join(ROOT, 'include')}"]
HIP_FLAGS = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in p.stdout.splitlines() if "packed-fp32-ops" not in l)
    if p.returncode != 0:
        raise RuntimeError(f"command failed ({p.returncode}): {' '.join(cmd)}\n{out}")
    return out


def build(verbose: bool = False, out: str | None = None, extra_flags=(), csrc: str | None = None) -> str:
    """Compile and link; `out`, `extra_flags` (e.g. -DQSIM_LDS_SWIZZLE=0) and
    `csrc` (another source directory) build a variant library elsewhere for
    comparisons."""
    CSRC_ = csrc or CSRC
    lib_out = out or LIB
    build_dir = BUILD if out is None else out + ".build"
    os.makedirs(build_dir, exist_ok=True)
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    clang = os.path.join(ROCM, "llvm", "bin", "clang++")
    jobs = []
    objs = []
    for src in HOST_SOURCES:
        path = os.path.join(CSRC_, src)
        if not os.path.exists(path):
            continue
        obj = os.path.join(build_dir, src + ".o")
        objs.append(obj)
        jobs.append([clang, *COMMON, f"-I{CSRC_}", *extra_flags, "-D__HIP_PLATFORM_AMD__", f"-I{os.path.join(ROCM, 'include')}",
                     "-pthread", "-c", path, "-o", obj])
    for src in DEVICE_SOURCES:
        path = os.path.join(CSRC_, src)
        obj = os.path.join(build_dir, src + ".o")
        objs.append(obj)
        jobs.append([hipcc, *HIP_FLAGS, *COMMON, f"-I{CSRC_}", *extra_flags, "-c", path, "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for out in ex.map(_run, jobs):
            if verbose and out.strip():
                print(out)
    tmp = lib_out + f".tmp{os.getpid()}"
    _run([hipcc, "--offload-arch=gfx950", "-shared", "-fPIC", "-pthread", "-o", tmp, *objs,
          f"-L{os.path.join(ROCM, 'lib')}", "-lamdhip64"])
    os.replace(tmp, lib_out)
    return lib_out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
