"""GPU tests of the bfloat16 trial of the mixed form (MEVP_MIXED_BF16): every
entry of the element matrices (reference basis and gradient tables, Jacobian
factors, quadrature weights times |J|, the local mass matrix's factors)
rounded to bfloat16, the arithmetic in float, the rest as in the mixed form.

The trial is measured, not expected to meet the mixed form's 1e-5: bfloat16
keeps 8 significant bits, so every matrix entry carries a relative rounding
error up to 2^-9 ~ 2e-3, and the per-field errors against the FP64 oracle are
of that order and above (logged by every test). What is asserted: the error
stays below TOLBF (a bound for an 8-bit operator, not a parity target), it is
far above the mixed form's (the rounding is really applied), the trial is
deterministic across launch strategies and tile shapes (they share its
arithmetic), and it rejects the configurations it does not build."""
import numpy as np
import pytest

from gpu_util import field_errors, gpu_run, log, oracle_run
from synth_inputs import make_domain, named_workload, random_state

pytestmark = pytest.mark.gpu

# per field, normwise: a bound for 8-bit element matrices (measured on one
# MI355X: at most 1.5e-2, S12 of the bilinear 10 km whole step; ~2e-3 over
# three subcycles at 256 x 256 and 2048 x 2048), not a parity target
TOLBF = 5e-2
TOLMIX = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_2402_00466_amd as M
    M.lib()


def _report(errs, what):
    log(f"{what}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    return errs


@pytest.mark.parametrize("perturb", [0.0, 0.1], ids=["parallelogram", "bilinear"])
def test_bf16_whole_run_10km(perturb):
    """One step of 100 subcycles on a 40 x 30 mesh of 10 km cells from rest:
    bf16 and mixed against the FP64 oracle, field by field."""
    d = make_domain(40, 30, 6, 1, seed=4001, h=10e3, perturb=perturb)
    vr, Sr = oracle_run(d, 1, 100)
    assert np.abs(vr).max() > 1e-3
    (vb, Sb), = gpu_run([d], 1, 100, precision="mixed_bf16", strategy="fused_pair")
    (vm, Sm), = gpu_run([d], 1, 100, precision="mixed", strategy="fused_pair")
    eb = _report(field_errors(vb, Sb, vr, Sr), f"bf16 40x30 perturb={perturb} 1x100")
    em = _report(field_errors(vm, Sm, vr, Sr), f"mixed 40x30 perturb={perturb} 1x100")
    assert all(v <= TOLMIX for v in em.values())
    assert all(v <= TOLBF for v in eb.values()), eb
    assert max(eb.values()) > 100 * max(em.values())


@pytest.mark.parametrize("name", ["256x256-dg2", "2048x2048-dg2", "2048x2048-dg2-bilinear"])
def test_bf16_few_subcycles_full_size(name):
    """Three subcycles from a seeded state at the workload's full size."""
    d, = named_workload(name)
    state = random_state(d.nx, d.ny, d.n_s, seed=99)
    vr, Sr = oracle_run(d, 1, 3, state=state)
    (vb, Sb), = gpu_run([d], 1, 3, precision="mixed_bf16", states=[state], strategy="fused_triple")
    eb = _report(field_errors(vb, Sb, vr, Sr), f"bf16 {name} 3 subcycles")
    assert all(v <= TOLBF for v in eb.values()), eb
    assert max(eb.values()) > 10 * TOLMIX


@pytest.mark.parametrize("perturb", [0.0, 0.1], ids=["parallelogram", "bilinear"])
def test_bf16_strategies_and_tiles_bitwise(perturb):
    """Every launch configuration of the trial gives the same bits (173 x 61
    mesh, ragged tiles, 7 subcycles from a seeded state)."""
    d = make_domain(173, 61, 6, 1, seed=61, h=3e3, perturb=perturb)
    state = random_state(d.nx, d.ny, d.n_s, seed=5)
    ref = None
    for strategy in ("fused", "fused_pair", "fused_triple"):
        for tile in ((16, 14), (16, 16), (32, 15), (13, 13)):
            (v, S), = gpu_run([d], 1, 7, precision="mixed_bf16", states=[state],
                              strategy=strategy, tile=tile)
            if ref is None:
                ref = (v, S)
            else:
                assert np.array_equal(v, ref[0]) and np.array_equal(S, ref[1]), (strategy, tile)


def test_bf16_rejects_what_it_does_not_build():
    import torch
    import paper_2402_00466_amd as M
    for dom in (M.Domain(8, 8, 3, 1), M.Domain(8, 8, 6, 3), M.Domain(8, 8, 8, 1)):
        with pytest.raises(M.MevpError) as ei:
            M.Context([dom], precision="mixed_bf16")
        assert ei.value.status == -1
    ctx = M.Context([M.Domain(8, 8, 6, 1)], precision="mixed_bf16")
    for strategy in ("two_phase", "persistent"):
        with pytest.raises(M.MevpError) as ei:
            ctx.set_strategy(strategy)
        assert ei.value.status == -1
    nodes = torch.zeros((2, 17 * 17), dtype=torch.float64, device="cuda")
    with pytest.raises(M.MevpError) as ei:
        ctx.set_geometry_cg2(0, nodes)
    assert ei.value.status == -1
    ctx.close()


def test_bf16_tuner_and_static_entry_agree():
    """The tuner's choice and mevp_step_static give the context path's bits."""
    import torch
    import paper_2402_00466_amd as M
    d = make_domain(45, 37, 6, 1, seed=9, h=10e3, perturb=0.1)
    state = random_state(d.nx, d.ny, d.n_s, seed=3)
    (v0, S0), = gpu_run([d], 1, 20, precision="mixed_bf16", states=[state], strategy="fused")
    (v1, S1), = gpu_run([d], 1, 20, precision="mixed_bf16", states=[state], strategy="tuned")
    assert np.array_equal(v0, v1) and np.array_equal(S0, S1)
    t = lambda a: torch.as_tensor(a, dtype=torch.float64).contiguous().cuda()
    v, S = t(state[0]), t(state[1])
    M.step_static(M.Domain(d.nx, d.ny, d.n_s, d.n_a), t(d.vertices), t(d.H), t(d.A), t(d.wind),
                  t(d.ocean), v, S, 20, precision="mixed_bf16")
    torch.cuda.synchronize()
    assert np.array_equal(v.cpu().numpy(), v0) and np.array_equal(S.cpu().numpy(), S0)
