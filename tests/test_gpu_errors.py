"""GPU tests of the error paths that need a device: out-of-order calls, the
device-side input and state checks, shape validation in the binding. Every
condition is forced from the host; no kernel faults or hangs."""
import math

import numpy as np
import pytest

from synth_inputs import make_domain

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def M():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_2402_00466_amd as M
    M.lib()
    return M


def test_step_before_inputs_is_state_error(M):
    ctx = M.Context([M.Domain(4, 4, 6, 1), M.Domain(3, 5, 6, 1)])
    d = make_domain(4, 4, 6, 1, seed=1, h=1e4)
    ctx.upload(0, d)  # domain 1 not set
    with pytest.raises(M.MevpError) as ei:
        ctx.step(1)
    assert ei.value.status == -4
    with pytest.raises(M.MevpError):
        ctx.subcycles(1)
    with pytest.raises(M.MevpError) as ei:
        ctx.subcycles(-1)
    assert ei.value.status == -1


def test_check_inputs_finds_nonfinite_and_inverted_cells(M):
    import torch
    d = make_domain(6, 5, 6, 1, seed=2, h=1e4)
    ctx = M.Context([M.Domain(6, 5, 6, 1)])
    ctx.upload(0, d)
    ctx.check_inputs()
    H = d.H.copy()
    H[0, 7] = math.nan
    ctx.set_fields(0, torch.as_tensor(H).cuda(), torch.as_tensor(d.A).cuda())
    with pytest.raises(M.MevpError) as ei:
        ctx.check_inputs()
    assert ei.value.status == -5
    ctx.set_fields(0, torch.as_tensor(d.H).cuda(), torch.as_tensor(d.A).cuda())
    ctx.check_inputs()
    V = d.vertices.copy()
    V[0, 8], V[0, 9] = V[0, 9], V[0, 8]  # swap two vertices: inverted cells
    ctx.set_geometry(0, torch.as_tensor(V).cuda())
    with pytest.raises(M.MevpError) as ei:
        ctx.check_inputs()
    assert ei.value.status == -5


def test_check_state_finds_nonfinite(M):
    import torch
    d = make_domain(5, 5, 6, 1, seed=3, h=1e4)
    for prec in ("fp64", "mixed"):
        ctx = M.Context([M.Domain(5, 5, 6, 1)], precision=prec)
        ctx.upload(0, d)
        ctx.step(2)
        ctx.check_state()
        v, S = ctx.get_state(0)
        S[1, 2, 3] = math.inf
        ctx.set_state(0, v, S)
        with pytest.raises(M.MevpError) as ei:
            ctx.check_state()
        assert ei.value.status == -5


def test_binding_rejects_bad_tensors(M):
    import torch
    ctx = M.Context([M.Domain(4, 3, 6, 1)])
    good = torch.zeros((2, 20), dtype=torch.float64, device="cuda")
    with pytest.raises(ValueError):
        ctx.set_geometry(0, good.float())          # wrong dtype
    with pytest.raises(ValueError):
        ctx.set_geometry(0, torch.zeros((2, 21), dtype=torch.float64, device="cuda"))  # shape
    with pytest.raises(ValueError):
        ctx.set_geometry(0, good.cpu())            # wrong device
    with pytest.raises(ValueError):
        ctx.set_geometry(0, torch.zeros((20, 2), dtype=torch.float64, device="cuda").t())  # strided
    with pytest.raises(IndexError):
        ctx.set_geometry(1, good)
    ctx.set_geometry(0, good)


def test_mixed_state_roundtrip_rounds_stress_to_float(M):
    import torch
    d = make_domain(4, 4, 6, 1, seed=9, h=1e4)
    ctx = M.Context([M.Domain(4, 4, 6, 1)], precision="mixed")
    ctx.upload(0, d)
    rng = np.random.default_rng(0)
    v = torch.as_tensor(rng.normal(size=(2, 81))).cuda()
    S = torch.as_tensor(rng.normal(size=(3, 6, 16)) * 1e3).cuda()
    ctx.set_state(0, v, S)
    v2, S2 = ctx.get_state(0)
    ctx.sync()
    assert torch.equal(v2, v)
    assert torch.equal(S2, S.float().double())
    # host pointers for S are refused in mixed mode (the rounding runs on the device)
    L = M.lib()
    import ctypes as C
    host = np.zeros((3, 6, 16))
    rc = L.mevp_set_state(ctx._h, 0, C.c_void_p(v.data_ptr()), host.ctypes.data_as(C.c_void_p))
    assert rc == -1
