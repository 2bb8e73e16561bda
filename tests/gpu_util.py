"""Helpers for the GPU parity tests: run the HIP path through the C ABI and the
FP64 oracle on the same seeded inputs, and compare field by field."""
from __future__ import annotations

import sys

import numpy as np


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def normwise(x, ref):
    """max |x - ref| / max |ref| (0 if both vanish)."""
    den = np.abs(ref).max()
    num = np.abs(x - ref).max()
    if den == 0.0:
        return float(num)
    return float(num / den)


def field_errors(v, S, vr, Sr):
    return {"vx": normwise(v[0], vr[0]), "vy": normwise(v[1], vr[1]),
            "S11": normwise(S[0], Sr[0]), "S12": normwise(S[1], Sr[1]),
            "S22": normwise(S[2], Sr[2])}


def gpu_run(domains, n_steps, n_sub, precision="fp64", states=None, params=None,
            subcycles_only=False, strategy="fused", tile=None):
    """Run every domain in ONE context; return [(v, S)] as numpy arrays.
    strategy="tuned": the launch configuration the autotuner picks for these
    domains (the one the benchmark times), chosen before the initial state is set."""
    import torch
    import paper_2402_00466_amd as M
    tuned = strategy == "tuned"
    ctx = M.Context([M.Domain(d.nx, d.ny, d.n_s, d.n_a) for d in domains], params=params,
                    precision=precision, strategy="fused" if tuned else strategy)
    if tile is not None:
        ctx.set_config(strategy, tile)
    for k, d in enumerate(domains):
        ctx.upload(k, d)
    if tuned:
        ctx.tune(n_trial=10)
        log(f"  tuned configuration: {ctx.get_config()}")
    for k, d in enumerate(domains):
        if states is not None:
            v, S = states[k]
            ctx.set_state(k, torch.as_tensor(v).cuda(), torch.as_tensor(S).cuda())
    for _ in range(n_steps):
        if subcycles_only:
            ctx.subcycles(n_sub)
        else:
            ctx.step(n_sub)
    out = []
    for k in range(len(domains)):
        v, S = ctx.get_state(k)
        out.append((v, S))
    ctx.sync()
    res = [(v.cpu().numpy(), S.cpu().numpy()) for v, S in out]
    ctx.close()
    return res


def oracle_mesh(d):
    """The oracle's mesh of a domain: isoparametric if it has CG2 node positions."""
    import oracle
    if getattr(d, "nodes", None) is not None:
        return oracle.Mesh(d.nx, d.ny, d.n_s, d.n_a, nodes=d.nodes)
    return oracle.Mesh(d.nx, d.ny, d.n_s, d.n_a, d.vertices)


def oracle_run(d, n_steps, n_sub, state=None, params=None):
    import oracle
    m = oracle_mesh(d)
    p = params or oracle.Params()
    v, S = (None, None) if state is None else state
    return m.run(p, d.H, d.A, d.wind, d.ocean, n_steps, n_sub, v=v, S=S)


def oracle_params(mp):
    """oracle.Params with the same values as a binding Params."""
    import dataclasses
    import oracle
    return oracle.Params(**dataclasses.asdict(mp))
