"""CPU tests of the C ABI: the library loads, exports every declared symbol, and
rejects bad arguments on the host before any device work (no compute calls)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def M():
    import paper_2402_00466_amd as M
    M.lib()
    return M


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "mevp.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mevp_[a-z0-9_]+)\s*\(", src)))


def test_exports_every_declared_symbol(M):
    syms = _declared_symbols()
    assert len(syms) >= 18
    L = C.CDLL(M.lib_path())
    for s in syms:
        assert hasattr(L, s), f"{s} declared in mevp.h but not exported"
    assert sorted(M.EXPORTS) == syms


def test_library_links_no_oracle_and_no_torch(M):
    """The product library is self-contained HIP: it must not depend on the oracle or torch."""
    import subprocess
    out = subprocess.run(["ldd", M.lib_path()], capture_output=True, text=True).stdout
    names = [line.split()[0] for line in out.splitlines() if line.strip()]
    assert not any("oracle" in n or "torch" in n or n.startswith("libc10") for n in names), names
    assert any(n.startswith("libamdhip64") for n in names), names


def test_default_params_match_paper_values(M):
    p = M.default_params()
    assert p.Pstar == 27500.0 and p.C == 20.0 and p.alpha == 300.0 and p.beta == 300.0
    assert p.dt == 120.0 and p.relax_form == 0
    assert M.Params() == p


def test_workspace_size_valid_and_monotone(M):
    D = M.Domain
    a = M.workspace_size([D(32, 32, 3, 1)])
    b = M.workspace_size([D(64, 32, 3, 1)])
    c = M.workspace_size([D(64, 32, 3, 1)], "mixed")
    e = M.workspace_size([D(64, 32, 6, 1), D(17, 5, 6, 1)])
    assert 0 < a < b and c < b and e > M.workspace_size([D(64, 32, 6, 1)])
    assert a % 256 == 0


@pytest.mark.parametrize("doms", [
    [(0, 4, 6, 1)], [(4, -1, 6, 1)], [(4, 4, 5, 1)], [(4, 4, 6, 2)], [(4, 4, 6, 1), (4, 4, 3, 1)],
    [(4, 4, 6, 1), (4, 4, 6, 3)], [(70000, 70000, 6, 1)]])
def test_workspace_size_rejects_bad_domains(M, doms):
    with pytest.raises(M.MevpError) as ei:
        M.workspace_size([M.Domain(*d) for d in doms])
    assert ei.value.status == -1


def test_null_and_empty_arguments(M):
    L = M.lib()
    out = C.c_size_t(0)
    assert L.mevp_workspace_size(None, 1, 0, C.byref(out)) == -1
    arr = (M.mevp.CDomain * 1)(M.mevp.CDomain(4, 4, 6, 1))
    assert L.mevp_workspace_size(arr, 0, 0, C.byref(out)) == -1
    assert L.mevp_workspace_size(arr, 1, 7, C.byref(out)) == -1   # bad precision
    assert L.mevp_workspace_size(arr, 1, 0, None) == -1
    assert L.mevp_default_params(None) == -1
    # every context call rejects a NULL context
    for f, args in [("mevp_set_geometry", (0, None)), ("mevp_set_fields", (0, None, None)),
                    ("mevp_set_forcing", (0, None, None)), ("mevp_set_state", (0, None, None)),
                    ("mevp_step", (1,)), ("mevp_begin_step", ()), ("mevp_subcycles", (1,)),
                    ("mevp_get_state", (0, None, None)), ("mevp_sync", ()),
                    ("mevp_check_inputs", ()), ("mevp_check_state", ())]:
        assert getattr(L, f)(None, *args) == -1, f
    L.mevp_destroy(None)  # no-op


def _create(M, params=None, ws=0x10000000, ws_bytes=None, doms=((8, 8, 6, 1),), prec=0):
    L = M.lib()
    arr = (M.mevp.CDomain * len(doms))(*[M.mevp.CDomain(*d) for d in doms])
    if ws_bytes is None:
        ws_bytes = M.workspace_size([M.Domain(*d) for d in doms])
    p = (params or M.Params()).to_c()
    h = C.c_void_p()
    return L.mevp_create(C.byref(p), prec, arr, len(doms), C.c_void_p(ws), C.c_size_t(ws_bytes),
                         None, C.byref(h))


@pytest.mark.parametrize("field,value", [("alpha", 0.0), ("dt", -1.0), ("DeltaMin", 0.0),
                                         ("DeltaMin", 1e-200),
                                         ("beta", -1.0), ("Pstar", float("nan")),
                                         ("C", float("inf")), ("rho_i", 0.0), ("relax_form", 2)])
def test_create_rejects_bad_params_before_device(M, field, value):
    p = M.Params()
    setattr(p, field, value)
    assert _create(M, params=p) == -1


def test_create_rejects_workspace_problems_before_device(M):
    assert _create(M, ws=0) == -1                 # NULL workspace
    assert _create(M, ws=0x10000000 + 8) == -1    # not 256-byte aligned
    need = M.workspace_size([M.Domain(8, 8, 6, 1)])
    assert _create(M, ws_bytes=need - 1) == -2    # too small
    assert _create(M, ws_bytes=1 << 20, doms=((8, 8, 6, 1), (8, 8, 3, 1))) == -1


def test_create_without_device_reports_device_error(M):
    """All host checks pass; with no GPU the first runtime call fails -> EDEVICE, never a crash."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a device is present; the fake workspace pointer must not reach it")
    assert _create(M) == -3


def test_status_strings(M):
    L = M.lib()
    for s, text in [(0, "ok"), (-1, "invalid argument"), (-2, "workspace too small"),
                    (-3, "device error"), (-4, "call out of order"),
                    (-5, "non-finite or invalid values"), (-6, "unsupported device"),
                    (-7, "internal self-check failed"), (-8, "host memory allocation failed")]:
        assert L.mevp_status_string(s).decode() == text
    assert L.mevp_status_string(99).decode() == "unknown status"
    assert L.mevp_version().decode().startswith("mevp-gfx950")


def test_binding_status_names_cover_the_header():
    """Every status the header declares has a name in the binding."""
    import re
    import paper_2402_00466_amd.mevp as mevp
    hdr = open(os.path.join(ROOT, "include", "mevp.h")).read()
    body = re.search(r"typedef enum \{(.*?)\} mevp_status;", hdr, re.S).group(1)
    declared = {int(v): k for k, v in re.findall(r"(MEVP_\w+) = (-?\d+)", body)}
    assert declared == mevp.STATUS


def test_binding_fails_loudly_without_library(M, monkeypatch, tmp_path):
    import paper_2402_00466_amd.mevp as mm
    monkeypatch.setattr(mm, "_lib", None)
    monkeypatch.setattr(mm._build, "LIB", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="not built"):
        mm.lib()


def test_binding_tiles_match_the_kernel_tile_shapes():
    """The binding's owned-tile list is the kernels' tile table (workgroup tiles
    including the one-element halo) minus the halo, in the same order."""
    import re
    import paper_2402_00466_amd.mevp as mevp
    src = open(os.path.join(ROOT, "paper_2402_00466_amd", "csrc", "mevp_internal.hpp")).read()
    m = re.search(r"kTileShapes\[kNumTileShapes\]\[2\] = \{(.*?)\};", src)
    shapes = [(int(a) - 1, int(b) - 1) for a, b in re.findall(r"\{(\d+), (\d+)\}", m.group(1))]
    n = int(re.search(r"kNumTileShapes = (\d+);", src).group(1))
    assert len(shapes) == n
    assert [tuple(t) for t in mevp.TILES] == shapes


def _step_static(M, doms=(8, 8, 6, 1), ptr=0x10000000, n=1, params=None, prec=0):
    L = M.lib()
    d = M.mevp.CDomain(*doms)
    p = (params or M.Params()).to_c()
    ptrs = [C.c_void_p(ptr)] * 7
    return L.mevp_step_static(C.byref(p), prec, C.byref(d), *ptrs, n, None)


def test_step_static_rejects_bad_arguments_before_device(M):
    L = M.lib()
    p = M.Params().to_c()
    d = M.mevp.CDomain(8, 8, 6, 1)
    ok = [C.c_void_p(0x10000000)] * 7
    for k in range(7):  # each NULL array
        ptrs = list(ok)
        ptrs[k] = None
        assert L.mevp_step_static(C.byref(p), 0, C.byref(d), *ptrs, 1, None) == -1
    assert L.mevp_step_static(None, 0, C.byref(d), *ok, 1, None) == -1
    assert L.mevp_step_static(C.byref(p), 0, None, *ok, 1, None) == -1
    assert L.mevp_step_static(C.byref(p), 3, C.byref(d), *ok, 1, None) == -1   # precision
    assert _step_static(M, n=-1) == -1
    assert _step_static(M, doms=(8, 8, 5, 1)) == -1
    bad = M.Params()
    bad.alpha = 0.0
    assert _step_static(M, params=bad) == -1


def test_step_static_rejects_domains_beyond_its_array(M):
    """The fixed device array holds ~1.1e5 elements at n_s = 6 in FP64: a
    larger domain is ENOMEM, decided on the host before any device call."""
    assert M.STATIC_SCRATCH_BYTES == 64 << 20
    hdr = open(os.path.join(ROOT, "include", "mevp.h")).read()
    assert "#define MEVP_STATIC_SCRATCH_BYTES ((size_t)64 << 20)" in hdr
    assert _step_static(M, doms=(512, 512, 6, 1)) == -2
    assert _step_static(M, doms=(400, 400, 6, 1)) == -2
    assert _step_static(M, doms=(512, 512, 3, 1), prec=1) == -2
    # the workspace of the context path is a bound from above on what it needs
    assert M.workspace_size([M.Domain(256, 256, 6, 1)]) < 2 * M.STATIC_SCRATCH_BYTES


def test_step_static_without_device_reports_device_error(M):
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a device is present; the fake pointers must not reach it")
    assert _step_static(M, doms=(64, 64, 6, 1)) == -3


def test_bf16_precision_sizes_and_limits(M):
    """The bfloat16 trial stores the stress in float like the mixed form and
    exists for n_s = 6, n_a = 1 only (EINVAL before any device call)."""
    D = M.Domain
    assert M.workspace_size([D(64, 32, 6, 1)], "mixed_bf16") == M.workspace_size([D(64, 32, 6, 1)], "mixed")
    for d in (D(8, 8, 3, 1), D(8, 8, 8, 1), D(8, 8, 6, 3)):
        with pytest.raises(M.MevpError) as ei:
            M.workspace_size([d], "mixed_bf16")
        assert ei.value.status == -1
    assert _step_static(M, doms=(8, 8, 3, 1), prec=2) == -1


_LOG_SCRIPT = r"""
import ctypes as C, sys
sys.path.insert(0, sys.argv[1])
import paper_2402_00466_amd as M
L = M.lib()
arr = (M.mevp.CDomain * 1)(M.mevp.CDomain(8, 8, 6, 1))
p = M.Params().to_c()
h = C.c_void_p()
need = M.workspace_size([M.Domain(8, 8, 6, 1)])
print(L.mevp_create(C.byref(p), 0, arr, 1, None, C.c_size_t(need), None, C.byref(h)))
print(L.mevp_create(C.byref(p), 0, arr, 1, C.c_void_p(0x10000000), C.c_size_t(need - 1), None,
                    C.byref(h)))
print(L.mevp_step(None, 1))
d = M.mevp.CDomain(8, 8, 6, 1)
print(L.mevp_step_static(C.byref(p), 0, C.byref(d), *([C.c_void_p(0x10000000)] * 7), -1, None))
"""


@pytest.mark.parametrize("level", [None, "0", "1"])
def test_log_env_reports_failing_calls_on_stderr(M, level):
    """MEVP_LOG=1 writes one line per failing call to stderr ("[mevp] call:
    status string (status n)"); unset or 0 writes nothing. Statuses are the
    same either way."""
    import subprocess
    import sys
    env = {k: v for k, v in os.environ.items() if k != "MEVP_LOG"}
    if level is not None:
        env["MEVP_LOG"] = level
    r = subprocess.run([sys.executable, "-c", _LOG_SCRIPT, ROOT], capture_output=True, text=True,
                       env=env, timeout=300)
    assert r.returncode == 0, r.stderr
    assert r.stdout.split() == ["-1", "-2", "-1", "-1"]
    lines = [x for x in r.stderr.splitlines() if x.startswith("[mevp]")]
    if level == "1":
        assert lines == ["[mevp] mevp_create: invalid argument (status -1)",
                         "[mevp] mevp_create: workspace too small (status -2)",
                         "[mevp] mevp_step: invalid argument (status -1)",
                         "[mevp] mevp_step_static: invalid argument (status -1)"]
    else:
        assert lines == []


def test_step_static_size_limit_matches_the_header(M):
    """The array holds about 610 B per element at n_s = 6 in FP64 and 470 B in
    mixed precision (64 MiB: ~1.1e5 / ~1.4e5 elements): the largest square
    domains that pass the host's size check are 330^2 and 375^2 (they then
    need a device), one size up is ENOMEM."""
    import torch
    if torch.cuda.device_count() > 0:
        pytest.skip("a device is present; the fake pointers must not reach it")
    assert _step_static(M, doms=(330, 330, 6, 1)) == -3
    assert _step_static(M, doms=(332, 332, 6, 1)) == -2
    assert _step_static(M, doms=(375, 375, 6, 1), prec=1) == -3
    assert _step_static(M, doms=(380, 380, 6, 1), prec=1) == -2
