#!/usr/bin/env python3
"""Benchmark of the mEVP momentum subcycle on one MI355X.

One benchmark step = one mEVP time step of the workload: the start-of-step
kernel (v^n, lumped masses, air stress) and n_sub = 100 subcycles of strain,
stress update, divergence and velocity update, with all inputs resident in HBM.
Prints ONE JSON line:
  value         element-subcycles per second (elements x subcycles x steps / time)
  roofline      the dominant kernel (element phase) against the HBM roofline,
                from its average duration measured with HIP events on the
                context's stream over the timed region
  cpu_baseline  the FP64 oracle on the host cores, on a bounded sample
  variants      the same measurement for mixed precision, the larger meshes
                and the 64-domain batch (one context, one launch per phase)

The default workload is 256 x 256 cells (2 km on a 512 km square), 6 DG
stress dofs, FP64, 100 subcycles per step, 10 steps.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
METRIC = "element-subcycles/sec (FP64 vs mixed/batched) + achieved HBM GB/s vs peak"
KERNEL_SOURCES = ["paper_2402_00466_amd/csrc/mevp_kernels.hip",
                  "paper_2402_00466_amd/csrc/mevp_ref.hpp",
                  "paper_2402_00466_amd/csrc/mevp_internal.hpp"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def alg_bytes(domains, precision):
    """Algorithmic HBM bytes of one launch of each phase (what it must move if
    nothing stays on chip between launches).
      element phase: S read + write (2 x 3 n_s words), H and A (2 n_a doubles)
                     per element; 2 doubles per vertex; v read, 2 doubles per node
      node phase:    v read + write (4 doubles) and 8 doubles of per-node
                     constants (v^n 2, ocean 2, air stress 2, M^H, m^A) per node
    The element forces passed between the phases are implementation scratch and
    not counted."""
    ws = 4 if precision == "mixed" else 8
    be = bn = 0
    for d in domains:
        ne, nn, nv = d.nx * d.ny, (2 * d.nx + 1) * (2 * d.ny + 1), (d.nx + 1) * (d.ny + 1)
        be += ne * (2 * 3 * d.n_s * ws + 2 * d.n_a * 8) + nv * 16 + nn * 16
        bn += nn * (32 + 64)
    return be, bn


def load_traffic(workload, precision):
    """HBM traffic of the element phase from committed rocprofv3 PMC summaries,
    if they were taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(f"{workload}/{precision}")
    except (ValueError, OSError):
        return None
    if not rec or rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


def run_gpu(domains, precision, steps, warmup, n_sub):
    import torch
    import paper_2402_00466_amd as M
    ctx = M.Context([M.Domain(d.nx, d.ny, d.n_s, d.n_a) for d in domains], precision=precision)
    for k, d in enumerate(domains):
        ctx.upload(k, d)
    ctx.check_inputs()
    for _ in range(warmup):
        ctx.step(n_sub)
    ctx.timing_enable(steps * n_sub + 8)
    ctx.sync()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    start.record(ctx.stream)
    for _ in range(steps):
        ctx.step(n_sub)
    stop.record(ctx.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = start.elapsed_time(stop)
    tim = ctx.timing_read()
    ctx.check_state()
    ctx.close()
    del ctx
    torch.cuda.synchronize()
    return ms, wall, tim


def measure(domains, precision, steps, warmup, n_sub, workload):
    ms, wall, tim = run_gpu(domains, precision, steps, warmup, n_sub)
    el_sub = sum(d.nx * d.ny for d in domains) * n_sub * steps
    value = el_sub / (ms * 1e-3)
    be, bn = alg_bytes(domains, precision)
    ne_cnt, ne_ms = tim["element"]
    nn_cnt, nn_ms = tim["node"]
    el_avg = ne_ms / max(ne_cnt, 1)
    nd_avg = nn_ms / max(nn_cnt, 1)
    achieved = be / (el_avg * 1e-3) / 1e9
    traffic = load_traffic(workload, precision)
    return {
        "value": value, "ms_per_step": ms / steps, "wall_s": wall,
        "kernels_ms": {"element_avg": el_avg, "node_avg": nd_avg,
                       "begin_step_avg": tim["begin_step"][1] / max(tim["begin_step"][0], 1),
                       "element_launches": ne_cnt, "node_launches": nn_cnt},
        "roofline": {"bound": "hbm", "kernel": "element_phase", "achieved": achieved,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "alg_bytes_per_launch": be,
                     "node_phase_achieved": bn / (nd_avg * 1e-3) / 1e9,
                     "subcycle_alg_GBs": (be + bn) / ((el_avg + nd_avg) * 1e-3) / 1e9},
    }


def cpu_baseline(domains, n_sub, budget_s):
    """The FP64 oracle as it stands, on the host: whole time steps of the first
    domain until ``budget_s`` of CPU time is spent (at least one)."""
    import oracle
    d = domains[0]
    m = oracle.Mesh(d.nx, d.ny, d.n_s, d.n_a, d.vertices)
    p = oracle.Params()
    v = S = None
    steps = 0
    t0 = time.perf_counter()
    while True:
        v, S = m.run(p, d.H, d.A, d.wind, d.ocean, 1, n_sub, v=v, S=S)
        steps += 1
        el = time.perf_counter() - t0
        if el >= budget_s or steps >= 10:
            break
    return {"value": d.nx * d.ny * n_sub * steps / el, "unit": "element-subcycles/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{steps} time step(s) x {n_sub} subcycles of {d.nx}x{d.ny} "
                      f"(n_s={d.n_s}), {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-sub", type=int, default=100)
    ap.add_argument("--workload", default="256x256-dg2")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): the mEVP subcycle "
              "here is single-GPU; see the sharding notes in DESIGN.md", file=sys.stderr)
        sys.exit(2)

    import torch
    from synth_inputs import named_workload
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    import paper_2402_00466_amd as M
    M.lib()

    log(f"workload {args.workload} {args.precision}: generating inputs")
    doms = named_workload(args.workload)
    head = measure(doms, args.precision, args.steps, args.warmup, args.n_sub, args.workload)
    log(f"headline {head['value']:.3e} element-subcycles/s, {head['ms_per_step']:.3f} ms/step")

    variants = {}
    if not args.no_variants:
        plan = [(args.workload, "mixed" if args.precision == "fp64" else "fp64", args.steps),
                ("1024x1024-dg2", "fp64", 3), ("1024x1024-dg2", "mixed", 3),
                ("2048x2048-dg2", "fp64", 2), ("2048x2048-dg2", "mixed", 2),
                ("batch64-dg2", "fp64", 2), ("batch64-dg2", "mixed", 2)]
        for wl, prec, st in plan:
            log(f"variant {wl} {prec} ({st} steps)")
            ds = doms if wl == args.workload else named_workload(wl)
            r = measure(ds, prec, st, 1, args.n_sub, wl)
            variants[f"{wl}/{prec}"] = {
                "value": r["value"], "ms_per_step": r["ms_per_step"], "steps": st,
                "elements": sum(d.nx * d.ny for d in ds),
                "element_phase_ms": r["kernels_ms"]["element_avg"],
                "node_phase_ms": r["kernels_ms"]["node_avg"],
                "roofline_frac": r["roofline"]["frac"],
                "achieved_GBs": r["roofline"]["achieved"],
                "subcycle_alg_GBs": r["roofline"]["subcycle_alg_GBs"]}
            log(f"  {r['value']:.3e} element-subcycles/s, element phase {r['roofline']['frac']:.3f} of HBM peak")
            del ds
        f64 = variants.get(f"{args.workload}/mixed")
        if f64 and args.precision == "fp64":
            variants["mixed_speedup_over_fp64"] = f64["value"] / head["value"]

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(doms, args.n_sub, args.cpu_budget)

    d0 = doms[0]
    line = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "element-subcycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "precision": args.precision,
                   "domains": len(doms), "elements": sum(d.nx * d.ny for d in doms),
                   "mesh": f"{d0.nx}x{d0.ny}", "n_s": d0.n_s, "n_a": d0.n_a,
                   "n_sub": args.n_sub, "step": "one mEVP time step (start-of-step kernel + n_sub subcycles)"},
        "roofline": head["roofline"],
        "kernels_ms": head["kernels_ms"],
        "cpu_baseline": cpu,
        "variants": variants,
        "kernel_hash": kernel_hash(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
