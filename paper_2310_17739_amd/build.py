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
          f"-L{os.path.join(ROCM, 'lib')}", "-lamdhip64", "-lrocprofiler-sdk-roctx"])
    os.replace(tmp, lib_out)
    return lib_out


def build_sanitized(out_dir: str | None = None) -> str:
    """Host sources with AddressSanitizer and UBSan (clang, shared sanitizer
    runtime), linked with the unchanged gfx950 kernels, into
    `out_dir`/libqsim.so: the CPU tests run against it to check the host
    logic (lowering, fusion, planning, packing, emulation, parser)."""
    out_dir = out_dir or os.path.join(HERE, "_asan")
    os.makedirs(out_dir, exist_ok=True)
    hipcc = os.path.join(ROCM, "bin", "hipcc")
    clang = os.path.join(ROCM, "llvm", "bin", "clang++")
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]
    jobs, objs = [], []
    for src in HOST_SOURCES:
        obj = os.path.join(out_dir, src + ".o")
        objs.append(obj)
        jobs.append([clang, *[f for f in COMMON if f != "-O3"], "-O1", *san, f"-I{CSRC}", "-D__HIP_PLATFORM_AMD__",
                     f"-I{os.path.join(ROCM, 'include')}", "-pthread", "-c", os.path.join(CSRC, src), "-o", obj])
    for src in DEVICE_SOURCES:
        obj = os.path.join(out_dir, src + ".o")
        objs.append(obj)
        jobs.append([hipcc, *HIP_FLAGS, *COMMON, f"-I{CSRC}", "-c", os.path.join(CSRC, src), "-o", obj])
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        list(ex.map(_run, jobs))
    lib = os.path.join(out_dir, "libqsim.so")
    _run([clang, "-shared", "-fPIC", "-pthread", "-fsanitize=address,undefined", "-shared-libsan", "-o", lib, *objs,
          f"-L{os.path.join(ROCM, 'lib')}", "-lamdhip64", "-lrocprofiler-sdk-roctx",
          f"-Wl,-rpath,{os.path.join(ROCM, 'lib')}"])
    return lib


def run_sanitized_tests(extra=()) -> int:
    """Build the sanitized library and oracle, then run the CPU tests
    (-m "not gpu") against them with the sanitizer runtime preloaded."""
    sys.path.insert(0, ROOT)
    import oracle
    lib = build_sanitized()
    olib = oracle.build_sanitized(os.path.join(HERE, "_asan", "liboracle.so"))
    rt = subprocess.run([os.path.join(ROCM, "llvm", "bin", "clang++"), "-print-file-name=libclang_rt.asan-x86_64.so"],
                        stdout=subprocess.PIPE, text=True, check=True).stdout.strip()
    if not os.path.isabs(rt):
        rt = subprocess.run([os.path.join(ROCM, "llvm", "bin", "clang++"), "--print-runtime-dir"],
                            stdout=subprocess.PIPE, text=True, check=True).stdout.strip() + "/libclang_rt.asan-x86_64.so"
    env = dict(os.environ, QSIM_LIB=lib, ORACLE_LIB=olib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:protect_shadow_gap=0:detect_odr_violation=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests"), "-q", "-m", "not gpu", "-p", "no:cacheprovider",
           *extra]
    return subprocess.call(cmd, env=env, cwd=ROOT)


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        sys.exit(run_sanitized_tests([a for a in sys.argv[1:] if a != "--sanitize"]))
    print(build(verbose="-v" in sys.argv))
