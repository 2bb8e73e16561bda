"""CPU check of the fused tile kernels' indexing (tests/index_check.hip).

The program is compiled by hipcc for the host only and walks every tile,
lane, element phase, node phase and node round of k_fused (one subcycle per
pass) and k_fused_multi (two and three) for every tile shape over domains with
ragged tails, one element wide and single elements, computing each index with
the kernels' own functions (paper_2402_00466_amd/csrc/mevp_index.hpp): LDS
reads and writes in bounds (missing elements' reads included), every summed
force from an element computed in that phase with the node as the expected
local node in ascending element order, every LDS velocity read written by the
node phase before it, the float-reciprocal division exact, and every node and
element stored exactly once over all tiles. No device is used."""
from __future__ import annotations

import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def test_tile_indexing_in_bounds_and_complete():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not installed")
    workdir = tempfile.mkdtemp(prefix="mevp_index_")
    try:
        exe = os.path.join(workdir, "index_check")
        subprocess.run([HIPCC, "--offload-arch=gfx950", "-O2", "-std=c++17",
                        "-I", os.path.join(ROOT, "include"),
                        "-I", os.path.join(ROOT, "paper_2402_00466_amd", "csrc"),
                        "-o", exe, os.path.join(ROOT, "tests", "index_check.hip")],
                       check=True, capture_output=True, text=True)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    finally:
        shutil.rmtree(workdir, ignore_errors=True)
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("ok "), r.stdout
    assert int(r.stdout.split()[1]) == 16 * 3 * 4  # domains x passes x tile shapes


# Plausible mistakes in the index header, each planted in a temporary copy
# that the check is compiled against: every one must make the check fail.
PLANTED = {
    "owned nodes one column short": ("r.ix1 = (x0 + TX >= nx) ? NX : r.ix0 + 2 * TX;",
                                     "r.ix1 = (x0 + TX >= nx) ? NX : r.ix0 + 2 * TX - 1;"),
    "phase range one element late": ("const int a = 2 * (ex0 + i + 1), b = 2 * (ey0 + i + 1);",
                                     "const int a = 2 * (ex0 + i + 2), b = 2 * (ey0 + i + 1);"),
    "phase range one element too far": ("const int c = 2 * (x0 + TX + K - 2 - i) + 1,",
                                        "const int c = 2 * (x0 + TX + K - 1 - i) + 1,"),
    "boundary column left out of a phase": ("r.ix0 = a > 0 ? a : 0;", "r.ix0 = a > 0 ? a : 1;"),
    "node column from the wrong width": ("dx = k - dy * w;", "dx = k - dy * (w - 1);"),
    "second and third force reads swapped": ("off[1] = base + b3 * NF + 1;\n  off[2] = base + c0 * NF + FW;",
                                             "off[1] = base + c0 * NF + FW;\n  off[2] = base + b3 * NF + 1;"),
    "local node row of the first read": ("const int b3 = two_y ? 6 : 3", "const int b3 = two_y ? 3 : 6"),
    "element-boundary test inverted in x": ("two_x = !(ix & 1);", "two_x = (ix & 1);"),
    "last strip as wide as the others": ("col = strip * j + off % w;", "col = strip * j + off % strip;"),
}


@pytest.mark.parametrize("name", sorted(PLANTED))
def test_planted_index_mistake_fails_the_check(name):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not installed")
    old, new = PLANTED[name]
    src = open(os.path.join(ROOT, "paper_2402_00466_amd", "csrc", "mevp_index.hpp")).read()
    assert src.count(old) == 1, name
    workdir = tempfile.mkdtemp(prefix="mevp_index_mut_")
    try:
        with open(os.path.join(workdir, "mevp_index.hpp"), "w") as f:
            f.write(src.replace(old, new))
        exe = os.path.join(workdir, "index_check")
        subprocess.run([HIPCC, "--offload-arch=gfx950", "--cuda-host-only", "-O2", "-std=c++17",
                        "-I", workdir, "-I", os.path.join(ROOT, "include"),
                        "-I", os.path.join(ROOT, "paper_2402_00466_amd", "csrc"),
                        "-o", exe, os.path.join(ROOT, "tests", "index_check.hip")],
                       check=True, capture_output=True, text=True)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    finally:
        shutil.rmtree(workdir, ignore_errors=True)
    assert r.returncode == 1 and r.stderr.startswith("FAIL "), (name, r.stdout, r.stderr[-300:])
