"""GPU parity on curved cells (isoparametric CG2 map, mevp_set_geometry_cg2)
against the FP64 oracle's isoparametric mesh (pinned in test_oracle_iso.py).
Tolerances as in test_gpu_parity.py: FP64 <= 1e-12, mixed <= 1e-5."""
import numpy as np
import pytest

from gpu_util import field_errors, gpu_run, log, oracle_mesh, oracle_run
from synth_inputs import make_domain, named_workload, random_state

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
TOLMIX = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_2402_00466_amd as M
    M.lib()


def _assert_close(errs, tol, what):
    log(f"{what}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, f"{what}: fields over {tol:g}: {bad}"


# (nx, ny, n_s, n_a, h, curved, ho_amp, n_steps, n_sub)
ISO_RUNS = [
    (12, 10, 6, 1, 10e3, 0.15, 0.0, 2, 20),
    (33, 17, 3, 1, 10e3, 0.10, 0.0, 1, 50),     # ragged tiles, 2x2 Gauss
    (40, 23, 6, 3, 12e3, 0.15, 0.3, 2, 30),     # n_a = 3, active clamps
    (9, 7, 8, 1, 10e3, 0.15, 0.0, 1, 40),       # n_s = 8
    (1, 5, 6, 1, 10e3, 0.10, 0.0, 1, 15),       # one element wide
]


@pytest.mark.parametrize("strategy", ["fused", "two_phase", "persistent", "fused_pair"])
@pytest.mark.parametrize("case", ISO_RUNS, ids=lambda c: "x".join(map(str, c[:4])))
def test_iso_whole_run_fp64(case, strategy):
    nx, ny, ns, na, h, cv, ho, steps, nsub = case
    d = make_domain(nx, ny, ns, na, seed=nx * 100 + ny + 7, h=h, curved=cv, ho_amp=ho)
    log(f"curved case {case} {strategy}")
    (v, S), = gpu_run([d], steps, nsub, strategy=strategy)
    vr, Sr = oracle_run(d, steps, nsub)
    assert np.abs(vr).max() > 1e-5
    _assert_close(field_errors(v, S, vr, Sr), TOL64, f"iso fp64 {nx}x{ny} ns={ns} na={na} {strategy}")


def test_iso_whole_run_mixed():
    d = make_domain(40, 23, 6, 3, seed=77, h=12e3, curved=0.15, ho_amp=0.3)
    (v, S), = gpu_run([d], 2, 30, precision="mixed")
    vr, Sr = oracle_run(d, 2, 30)
    _assert_close(field_errors(v, S, vr, Sr), TOLMIX, "iso mixed 40x23")


@pytest.mark.parametrize("precision,tol", [("fp64", TOL64), ("mixed", TOLMIX)])
@pytest.mark.parametrize("name", ["256x256-dg2-iso", "1024x1024-dg2-iso"])
def test_iso_few_subcycles_full_size(name, precision, tol):
    d, = named_workload(name)
    state = random_state(d.nx, d.ny, d.n_s, seed=99)
    log(f"workload {name} {precision}: 3 subcycles from a seeded state")
    (v, S), = gpu_run([d], 1, 3, precision=precision, states=[state])
    vr, Sr = oracle_run(d, 1, 3, state=state)
    _assert_close(field_errors(v, S, vr, Sr), tol, f"{name} {precision}")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_iso_launch_configs_agree_bitwise(precision):
    d = make_domain(173, 61, 6, 1, seed=62, h=2e3, curved=0.15)
    state = random_state(d.nx, d.ny, d.n_s, seed=5)
    ref = gpu_run([d], 2, 25, precision=precision, states=[state])[0]
    for strategy, tile in [("two_phase", None), ("fused", (16, 16)), ("fused", (32, 15)),
                           ("persistent", (16, 14)), ("fused_pair", (16, 14)),
                           ("fused_triple", (16, 16)), ("fused_pair", (13, 13))]:
        got = gpu_run([d], 2, 25, precision=precision, states=[state], strategy=strategy,
                      tile=tile)[0]
        log(f"iso {strategy} {tile} vs fused (16, 14), {precision}")
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]), (strategy, tile)


def test_mixed_geometry_kinds_batched_equal_solo_and_oracle():
    """Parallelogram, bilinear and curved domains in one context: three element
    kernels per launch; each domain equals its solo run bitwise and the oracle."""
    doms = [make_domain(30, 20, 6, 1, seed=1, h=10e3),
            make_domain(25, 33, 6, 1, seed=2, h=10e3, perturb=0.1),
            make_domain(21, 19, 6, 1, seed=3, h=10e3, curved=0.15),
            make_domain(17, 9, 6, 1, seed=4, h=10e3)]
    for strategy in ("fused", "fused_triple", "two_phase"):
        batched = gpu_run(doms, 2, 15, strategy=strategy)
        for k, d in enumerate(doms):
            (v, S), = gpu_run([d], 2, 15)
            assert np.array_equal(v, batched[k][0]) and np.array_equal(S, batched[k][1]), (strategy, k)
    for k, d in enumerate(doms):
        vr, Sr = oracle_run(d, 2, 15)
        _assert_close(field_errors(*batched[k], vr, Sr), TOL64, f"kinds batch domain {k}")


def test_iso_advection_matches_oracle():
    import torch
    import paper_2402_00466_amd as M
    d = make_domain(23, 17, 6, 3, seed=9, h=2e3, curved=0.15, ho_amp=0.2)
    state = random_state(d.nx, d.ny, d.n_s, seed=4, v_scale=0.3)
    ctx = M.Context([M.Domain(d.nx, d.ny, d.n_s, d.n_a)])
    ctx.upload(0, d)
    ctx.set_state(0, torch.as_tensor(state[0]).cuda(), torch.as_tensor(state[1]).cuda())
    m = oracle_mesh(d)
    H, A = d.H, d.A
    for _ in range(3):
        ctx.advect()
        H, A = m.advect(ctx.params.dt, state[0], H, A)
    Hg, Ag = ctx.get_fields(0)
    ctx.sync()
    eh = np.abs(Hg.cpu().numpy() - H).max() / np.abs(H).max()
    ea = np.abs(Ag.cpu().numpy() - A).max() / np.abs(A).max()
    log(f"iso advection: H {eh:.2e} A {ea:.2e}")
    assert np.abs(H - d.H).max() > 1e-6  # the fields moved
    assert eh <= 1e-13 and ea <= 1e-13


def test_geometry_kind_switches_with_the_last_setter():
    """set_geometry_cg2 then set_geometry on the same domain: the vertex geometry
    wins (equal bitwise to a context that only had the vertices), and back."""
    import torch
    import paper_2402_00466_amd as M
    dc = make_domain(20, 14, 6, 1, seed=5, h=10e3, curved=0.15)
    dv = make_domain(20, 14, 6, 1, seed=5, h=10e3, perturb=0.1)
    ref_v = gpu_run([dv], 1, 20)[0]
    ref_c = gpu_run([dc], 1, 20)[0]
    ctx = M.Context([M.Domain(20, 14, 6, 1)])
    ctx.upload(0, dc)
    ctx.set_geometry(0, torch.as_tensor(dv.vertices).cuda())
    ctx.step(20)
    v, S = ctx.get_state(0)
    ctx.sync()
    assert np.array_equal(v.cpu().numpy(), ref_v[0]) and np.array_equal(S.cpu().numpy(), ref_v[1])
    ctx2 = M.Context([M.Domain(20, 14, 6, 1)])
    ctx2.upload(0, dv)
    ctx2.set_geometry_cg2(0, torch.as_tensor(dc.nodes).cuda())
    ctx2.step(20)
    v2, S2 = ctx2.get_state(0)
    ctx2.sync()
    assert np.array_equal(v2.cpu().numpy(), ref_c[0]) and np.array_equal(S2.cpu().numpy(), ref_c[1])
