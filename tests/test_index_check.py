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
