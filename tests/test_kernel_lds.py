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


@pytest.mark.skipif(not (tool("bin", "hipcc") and tool("llvm", "bin", "clang-offload-bundler")
                         and tool("llvm", "bin", "llvm-readelf")), reason="ROCm tools missing")
def test_tile_kernel_has_no_static_lds(tmp_path):
    obj, co = tmp_path / "dev.o", tmp_path / "gfx950.co"
    subprocess.run([tool("bin", "hipcc"), "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
                    "-packed-fp32-ops", "-O3", "-std=c++17", f"-I{os.path.join(ROOT, 'include')}",
                    f"-I{CSRC}", "--offload-device-only", "-c", os.path.join(CSRC, "kernels.hip"),
                    "-o", str(obj)], check=True, capture_output=True)
    subprocess.run([tool("llvm", "bin", "clang-offload-bundler"), "--unbundle", "--type=o",
                    f"--input={obj}", "--targets=hipv4-amdgcn-amd-amdhsa--gfx950", f"--output={co}"],
                   check=True, capture_output=True)
    notes = subprocess.run([tool("llvm", "bin", "llvm-readelf"), "--notes", str(co)], check=True,
                           capture_output=True, text=True).stdout
    sizes, g = {}, None
    for line in notes.splitlines():
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
