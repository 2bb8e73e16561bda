"""GPU parity of the DG upwind advection of H and A (mevp_advect) with the
oracle, and of a whole time step (advection, then the momentum subcycles)."""
import numpy as np
import pytest

from gpu_util import field_errors, log, normwise
from synth_inputs import make_domain, random_state

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


CASES = [(23, 17, 6, 1, 0.0), (23, 17, 6, 3, 0.1), (40, 9, 6, 6, 0.15), (1, 1, 6, 3, 0.0),
         (300, 2, 3, 1, 0.0), (33, 33, 8, 6, 0.1)]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "x".join(map(str, c[:4])))
def test_advection_matches_oracle(M, case):
    import torch
    import oracle
    nx, ny, ns, na, pert = case
    d = make_domain(nx, ny, ns, na, seed=77 + nx, h=3e3, perturb=pert, ho_amp=0.2)
    v, S = random_state(nx, ny, ns, seed=5, v_scale=0.5)
    ctx = M.Context([M.Domain(nx, ny, ns, na)])
    ctx.upload(0, d)
    ctx.set_state(0, torch.as_tensor(v).cuda(), torch.as_tensor(S).cuda())
    m = oracle.Mesh(nx, ny, ns, na, d.vertices)
    H, A = d.H, d.A
    for k in range(3):
        ctx.advect()
        H, A = m.advect(120.0, v, H, A)
        Hg, Ag = ctx.get_fields(0)
        ctx.sync()
        eh, ea = normwise(Hg.cpu().numpy(), H), normwise(Ag.cpu().numpy(), A)
        log(f"advection {case} step {k}: H {eh:.2e} A {ea:.2e}")
        assert eh <= 1e-13 and ea <= 1e-13
    assert normwise(H, d.H) > 1e-6  # the fields moved


def test_batched_advection_and_full_step(M):
    """Two domains in one context: advection then 20 subcycles, three time
    steps, against the oracle doing the same."""
    import torch
    import oracle
    doms = [make_domain(18, 14, 6, 3, seed=5, h=10e3, ho_amp=0.1),
            make_domain(9, 21, 6, 3, seed=6, h=10e3, perturb=0.1)]
    ctx = M.Context([M.Domain(d.nx, d.ny, d.n_s, d.n_a) for d in doms])
    for k, d in enumerate(doms):
        ctx.upload(k, d)
    for _ in range(3):
        ctx.advect()
        ctx.step(20)
    p = oracle.Params()
    for k, d in enumerate(doms):
        m = oracle.Mesh(d.nx, d.ny, d.n_s, d.n_a, d.vertices)
        v = np.zeros((2, m.nn))
        S = np.zeros((3, d.n_s, m.ne))
        H, A = d.H, d.A
        for _ in range(3):
            H, A = m.advect(p.dt, v, H, A)
            v, S = m.step(p, H, A, d.wind, d.ocean, v, S, 20)
        vg, Sg = ctx.get_state(k)
        Hg, Ag = ctx.get_fields(k)
        ctx.sync()
        errs = field_errors(vg.cpu().numpy(), Sg.cpu().numpy(), v, S)
        errs["H"] = normwise(Hg.cpu().numpy(), H)
        errs["A"] = normwise(Ag.cpu().numpy(), A)
        log(f"domain {k}: " + " ".join(f"{a}={b:.2e}" for a, b in errs.items()))
        assert max(errs.values()) <= 1e-12
