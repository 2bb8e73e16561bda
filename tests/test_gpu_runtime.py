"""GPU tests of the runtime around the kernels: graph replay of a time step,
the autotuner and its cache, kernel timing."""
import numpy as np
import pytest

from gpu_util import gpu_run, log
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


def _ctx(M, d, **kw):
    ctx = M.Context([M.Domain(d.nx, d.ny, d.n_s, d.n_a)], **kw)
    ctx.upload(0, d)
    return ctx


def _state(ctx):
    v, S = ctx.get_state(0)
    ctx.sync()
    return v.cpu().numpy(), S.cpu().numpy()


@pytest.mark.parametrize("strategy", ["fused", "fused_pair", "fused_triple"])
@pytest.mark.parametrize("n_sub", [10, 7])
def test_graph_replays_match_eager(M, n_sub, strategy):
    """Graph replay of mevp_step (even and odd n_sub: one or two captured graphs),
    with eager work and host synchronisation between the replays: every step's
    result equals the eagerly launched one bitwise; a parameter change in
    between drops the graphs and is honoured."""
    d = make_domain(50, 37, 6, 1, seed=11, h=3e3)
    g = _ctx(M, d, strategy=strategy)
    e = _ctx(M, d, strategy=strategy)
    e.set_graph(False)
    for k in range(5):
        if k == 3:
            for c in (g, e):
                c.set_params(M.Params(alpha=250.0))
        g.step(n_sub)
        e.step(n_sub)
        vg, Sg = _state(g)   # eager work + sync between replays
        ve, Se = _state(e)
        assert np.array_equal(vg, ve) and np.array_equal(Sg, Se), k
    # eager subcycles on the graph context continue from the replayed state
    g.subcycles(3)
    e.subcycles(3)
    assert all(np.array_equal(a, b) for a, b in zip(_state(g), _state(e)))


def test_tune_keeps_state_and_result(M, tmp_path):
    d = make_domain(64, 40, 6, 1, seed=12, h=2e3)
    state = random_state(d.nx, d.ny, d.n_s, seed=3)
    import torch
    ctx = _ctx(M, d)
    ctx.set_state(0, torch.as_tensor(state[0]).cuda(), torch.as_tensor(state[1]).cuda())
    cache = tmp_path / "tune.txt"
    strategy, tile = ctx.tune(n_trial=5, cache_path=str(cache))
    log(f"tuned: {strategy} {tile}")
    assert strategy in M.STRATEGIES and tuple(tile) in M.TILES
    assert ctx.get_config() == (strategy, tuple(tile))
    v, S = _state(ctx)
    assert np.array_equal(v, state[0]) and np.array_equal(S, state[1])
    ctx.step(20)
    tuned = _state(ctx)
    ref = gpu_run([d], 1, 20, states=[state])[0]
    assert np.array_equal(tuned[0], ref[0]) and np.array_equal(tuned[1], ref[1])
    # the cache answers without timing and names the same configuration
    lines = cache.read_text().split("\n")
    assert lines[0].startswith("gfx950/fp64/ns6/na1/dom1/el2560/max64x40/geo2560.0.0 ")
    ctx2 = _ctx(M, d)
    assert ctx2.tune(n_trial=5, cache_path=str(cache)) == (strategy, tuple(tile))


def test_timing_counts_launches(M):
    d = make_domain(20, 20, 6, 1, seed=13, h=5e3)
    ctx = _ctx(M, d)
    ctx.timing_enable(64)
    ctx.step(10)
    t = ctx.timing_read()
    assert t["element"][0] == 10 and t["begin_step"][0] == 1 and t["node"][0] == 0
    assert t["element"][1] > 0
    ctx.set_strategy("two_phase")
    ctx.step(4)
    t = ctx.timing_read()
    assert t["element"][0] == 4 and t["node"][0] == 4
    ctx.timing_enable(0)


@pytest.mark.parametrize("kind", ["parallelogram", "bilinear", "curved", "parallelogram+bilinear"])
def test_launch_depth_matches_launches(M, kind):
    """mevp_get_launch_depth reports what a call actually launches: 10 subcycles
    take 10 / depth launches plus one for the remainder (one launch for the
    persistent strategy when it runs the whole call)."""
    d0 = make_domain(20, 18, 6, 1, seed=21, h=5e3,
                     perturb=0.1 if kind == "bilinear" else 0.0,
                     curved=0.1 if kind == "curved" else 0.0)
    doms = [d0]
    if kind == "parallelogram+bilinear":
        doms.append(make_domain(15, 11, 6, 1, seed=22, h=5e3, perturb=0.1))
    ctx = M.Context([M.Domain(d.nx, d.ny, d.n_s, d.n_a) for d in doms])
    for k, d in enumerate(doms):
        ctx.upload(k, d)
    most = {"parallelogram": 3, "bilinear": 2, "curved": 1, "parallelogram+bilinear": 2}[kind]
    expect = {"fused": 1, "two_phase": 1, "fused_pair": min(2, most), "fused_triple": most,
              "persistent": 1 if kind == "parallelogram+bilinear" else 0}
    ctx.set_graph(False)
    for strategy, depth in expect.items():
        ctx.set_config(strategy, (16, 14))
        assert ctx.launch_depth() == depth, strategy
        ctx.timing_enable(64)
        ctx.subcycles(10)
        n_launch = ctx.timing_read()["element"][0]
        ctx.timing_enable(0)
        want = 1 if depth == 0 else 10 // depth + (1 if depth > 1 and 10 % depth else 0)
        log(f"{kind} {strategy}: depth {depth}, {n_launch} launches for 10 subcycles")
        assert n_launch == want, (strategy, n_launch, want)
    ctx.sync()
    ctx.close()


_LOG_RUN = r"""
import hashlib, sys
sys.path.insert(0, sys.argv[1])
import torch
torch.cuda.set_device(0)
import paper_2402_00466_amd as M
from synth_inputs import make_domain
d = make_domain(40, 30, 6, 1, seed=13, h=2e3)
ctx = M.Context([M.Domain(d.nx, d.ny, d.n_s, d.n_a)])
ctx.upload(0, d)
ctx.tune(n_trial=3)
ctx.step(10)
v, S = ctx.get_state(0)
ctx.sync()
print(hashlib.sha256(v.cpu().numpy().tobytes() + S.cpu().numpy().tobytes()).hexdigest())
"""


def test_log_env_traces_create_tune_and_capture(M):
    """MEVP_LOG=2 writes the context, every tuner trial and the choice, the
    configurations set and the captured step graph to stderr; the state after a
    tuned step is the same with logging off (in a process of its own each, as
    the variable is read once per process)."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    runs = []
    for level in (None, "2"):
        env = {k: v for k, v in os.environ.items() if k != "MEVP_LOG"}
        if level:
            env["MEVP_LOG"] = level
        log(f"child process, MEVP_LOG={level}")
        r = subprocess.run([sys.executable, "-c", _LOG_RUN, root], capture_output=True,
                           text=True, env=env, timeout=240)
        assert r.returncode == 0, r.stderr[-3000:]
        runs.append(r)
    assert runs[0].stdout == runs[1].stdout
    assert "[mevp]" not in runs[0].stderr
    lines = [x for x in runs[1].stderr.splitlines() if x.startswith("[mevp]")]
    assert lines[0].startswith("[mevp] create: 1 domain(s), 1200 elements, "), lines[:3]
    assert "fp64, n_s 6, n_a 1" in lines[0]
    trials = [x for x in lines if x.startswith("[mevp] tune: ") and x.endswith(" ms for 3 subcycles")]
    assert len(trials) == 3 * len(M.TILES) + 1, trials   # fused, pair, triple per tile; two-phase
    chose = [x for x in lines if " chose " in x]
    assert len(chose) == 1 and chose[0].startswith("[mevp] tune: gfx950/fp64/ns6/na1/dom1/el1200/")
    assert any(x.startswith("[mevp] config: ") for x in lines)
    assert any(x.startswith("[mevp] step: graph captured (start of step + 10 subcycles, ")
               for x in lines)
    assert not any("status" in x for x in lines), lines
