"""Host-only check of the tile kernel's code object: it must declare no
static LDS, since its tile starts at LDS byte 0 and every other LDS region
is addressed from there.  (A private array indexed at run time can be moved
into LDS by the compiler; the library then refuses to start.)

The kernels are compiled for gfx950 device code only and the group segment
size of every k_tile instance is read from the code object's metadata.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2310_17739_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def tool(*parts):
    p = os.path.join(ROCM, *parts)
    return p if os.path.exists(p) else None


HAVE_TOOLS = bool(tool("bin", "hipcc") and tool("llvm", "bin", "clang-offload-bundler")
                  and tool("llvm", "bin", "llvm-readelf"))


@pytest.fixture(scope="module")
def kernel_notes(tmp_path_factory):
    """Metadata notes of the gfx950 code object of kernels.hip."""
    tmp = tmp_path_factory.mktemp("co")
    obj, co = tmp / "dev.o", tmp / "gfx950.co"
    subprocess.run([tool("bin", "hipcc"), "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                    "-packed-fp32-ops", "-O3", "-std=c++17", f"-I{os.path.join(ROOT, 'include')}",
                    f"-I{CSRC}", "--offload-device-only", "-c", os.path.join(CSRC, "kernels.hip"),
                    "-o", str(obj)], check=True, capture_output=True)
    subprocess.run([tool("llvm", "bin", "clang-offload-bundler"), "--unbundle", "--type=o",
                    f"--input={obj}", "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={co}"],
                   check=True, capture_output=True)
    return subprocess.run([tool("llvm", "bin", "llvm-readelf"), "--notes", str(co)], check=True,
                          capture_output=True, text=True).stdout


@pytest.mark.skipif(not HAVE_TOOLS, reason="ROCm tools missing")
def test_tile_kernel_has_no_static_lds(kernel_notes):
    sizes, g = {}, None
    for line in kernel_notes.splitlines():
        m = re.search(r"\.group_segment_fixed_size:\s+(\d+)", line)
        if m:
            g = int(m.group(1))
        m = re.search(r"^\s+\.name:\s+(\S+)", line)
        if m and g is not None:
            sizes[m.group(1)] = g
            g = None
    tiles = {k: v for k, v in sizes.items() if "k_tile" in k}
    assert len(tiles) == 28, sorted(tiles)
    assert all(v == 0 for v in tiles.values()), {k: v for k, v in tiles.items() if v}


@pytest.mark.skipif(not HAVE_TOOLS, reason="ROCm tools missing")
def test_default_tile_kernels_keep_two_workgroups_per_cu(kernel_notes):
    """The complex64 tile kernels of the default plans (512 threads, 8 or 16
    elements per thread: 12- and 13-qubit tiles) must fit 128 VGPRs, so that
    a CU holds two of their 8-wave workgroups (4 waves per SIMD); code
    compiled into them for other cases (in-tile measurements) must not raise
    their registers.  The complex128 default (256 threads, 16 elements) must
    fit 256 VGPRs (two 4-wave workgroups)."""
    vgprs, name = {}, None
    for line in kernel_notes.splitlines():
        m = re.search(r"^\s+\.name:\s+(\S+)", line)
        if m:
            name = m.group(1)
        m = re.search(r"\.vgpr_count:\s+(\d+)", line)
        if m and name is not None:
            vgprs[name] = int(m.group(1))
            name = None
    limits = {"_ZN2qk6k_tileIfLi3ELi512EEEv": 128, "_ZN2qk6k_tileIfLi4ELi512EEEv": 128,
              "_ZN2qk6k_tileIdLi4ELi256EEEv": 256}
    for prefix, lim in limits.items():
        got = [v for k, v in vgprs.items() if k.startswith(prefix)]
        assert len(got) == 1, (prefix, sorted(vgprs))
        assert got[0] <= lim, (prefix, got[0], lim)
