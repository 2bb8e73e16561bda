"""The oracle's pins run against an AddressSanitizer + UndefinedBehaviorSanitizer
build of the oracle (host code only: the oracle is plain C on the CPU).

The oracle is compiled with its own flags plus -fsanitize=address,undefined
-fno-sanitize-recover=all into a temporary library, and every pin file runs
against it in a subprocess (``oracle.ENV_LIB`` selects the library; the
sanitizer runtime is preloaded because the Python interpreter is not
instrumented). Any out-of-bounds access, use after free or undefined
operation in the oracle aborts that run, so the test fails."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["tests/test_oracle_tables.py", "tests/test_oracle_pins.py",
             "tests/test_oracle_composition.py", "tests/test_brute_2x2.py",
             "tests/test_oracle_iso.py", "tests/test_oracle_advection.py"]


def _asan_runtime():
    path = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                          text=True).stdout.strip()
    return path if path and os.path.isabs(path) and os.path.exists(path) else None


def test_oracle_pins_under_address_and_undefined_behaviour_sanitizers():
    import oracle.build as ob
    rt = _asan_runtime()
    if rt is None:
        pytest.skip("gcc's AddressSanitizer runtime is not installed")
    workdir = tempfile.mkdtemp(prefix="mevp_oracle_san_")
    try:
        lib = os.path.join(workdir, "liboracle_san.so")
        ob.build(lib=lib, extra=("-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                                 "-fno-omit-frame-pointer", "-g"))
        env = dict(os.environ, MEVP_ORACLE_LIB=lib, LD_PRELOAD=rt, OMP_NUM_THREADS="2",
                   ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            "-m", "not gpu"] + PIN_FILES, cwd=ROOT, env=env, capture_output=True,
                           text=True, timeout=1200)
    finally:
        shutil.rmtree(workdir, ignore_errors=True)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert " passed" in r.stdout and "ERROR: AddressSanitizer" not in r.stderr, tail
    assert "runtime error:" not in r.stderr, tail
