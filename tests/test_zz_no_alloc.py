"""GPU tests of mevp_step_static, the entry point that allocates nothing: its
output against the context path (mevp_create + set_* + mevp_step +
mevp_get_state) on the same inputs, on two calls in a row, the second with a
smaller domain (the device array it works in keeps the first call's
contents)."""
import numpy as np
import pytest

from gpu_util import log
from synth_inputs import make_domain

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    import paper_2402_00466_amd as M
    M.lib()


def _state(d, seed):
    """A seeded non-trivial state (velocity ~0.1 m/s, stress ~1e4 N/m)."""
    rng = np.random.default_rng(seed)
    nn, ne = (2 * d.nx + 1) * (2 * d.ny + 1), d.nx * d.ny
    return 0.1 * rng.standard_normal((2, nn)), 1e4 * rng.standard_normal((3, d.n_s, ne))


def _context(d, v0, S0, n_sub, precision):
    import torch
    import paper_2402_00466_amd as M
    ctx = M.Context([M.Domain(d.nx, d.ny, d.n_s, d.n_a)], precision=precision)
    ctx.upload(0, d)
    ctx.set_state(0, torch.as_tensor(v0).cuda(), torch.as_tensor(S0).cuda())
    ctx.step(n_sub)
    v, S = ctx.get_state(0)
    ctx.sync()
    out = v.cpu().numpy(), S.cpu().numpy()
    ctx.close()
    return out


def _static(d, v0, S0, n_sub, precision):
    import torch
    import paper_2402_00466_amd as M
    t = lambda a: torch.as_tensor(a, dtype=torch.float64).contiguous().cuda()
    v, S = t(v0), t(S0)
    M.step_static(M.Domain(d.nx, d.ny, d.n_s, d.n_a), t(d.vertices), t(d.H), t(d.A), t(d.wind),
                  t(d.ocean), v, S, n_sub, precision=precision)
    torch.cuda.synchronize()
    return v.cpu().numpy(), S.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("n_s,n_a,perturb", [(6, 1, 0.0), (6, 1, 0.2), (3, 1, 0.0), (8, 1, 0.0),
                                             (6, 3, 0.2)])
def test_static_matches_context_on_two_calls(precision, n_s, n_a, perturb):
    """Two calls in a row (a 45 x 37 domain, then a 19 x 11 one), each equal
    bit for bit to the context path; parallelogram and bilinear cells."""
    for k, (nx, ny, n_sub) in enumerate([(45, 37, 20), (19, 11, 7)]):
        d = make_domain(nx, ny, n_s, n_a, seed=700 + k, h=10e3, perturb=perturb,
                        ho_amp=0.1 if n_a > 1 else 0.0)
        v0, S0 = _state(d, 800 + k)
        log(f"call {k}: {nx}x{ny} n_s={n_s} n_a={n_a} perturb={perturb} {precision} {n_sub} subcycles")
        vr, Sr = _context(d, v0, S0, n_sub, precision)
        v, S = _static(d, v0, S0, n_sub, precision)
        assert np.abs(vr).max() > 1e-3
        assert np.array_equal(v, vr), np.abs(v - vr).max()
        assert np.array_equal(S, Sr), np.abs(S - Sr).max()


def test_static_zero_subcycles_and_too_large():
    """n_subcycles = 0 returns the state as the context path does; a domain
    beyond the array is ENOMEM and leaves the caller's state untouched."""
    import torch
    import paper_2402_00466_amd as M
    d = make_domain(9, 7, 6, 1, seed=5, h=10e3)
    v0, S0 = _state(d, 6)
    for precision in ("fp64", "mixed"):
        vr, Sr = _context(d, v0, S0, 0, precision)
        v, S = _static(d, v0, S0, 0, precision)
        assert np.array_equal(v, vr) and np.array_equal(S, Sr)
    big = M.Domain(400, 400, 6, 1)
    z = lambda *s: torch.zeros(s, dtype=torch.float64, device="cuda")
    v = torch.ones((2, big.nn), dtype=torch.float64, device="cuda")
    with pytest.raises(M.MevpError) as ei:
        M.step_static(big, z(2, big.nv), z(1, big.ne), z(1, big.ne), z(2, big.nn), z(2, big.nn),
                      v, z(3, 6, big.ne), 5)
    assert ei.value.status == -2
    torch.cuda.synchronize()
    assert bool((v == 1).all())
