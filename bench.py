#!/usr/bin/env python3
"""Benchmark of the mEVP momentum subcycle on one MI355X.

One benchmark step = one mEVP time step of the workload: the start-of-step
kernel (v^n, lumped masses, air stress) and n_sub = 100 subcycles of strain,
stress update, divergence and velocity update, with all inputs resident in HBM.
Prints ONE JSON line:
  value         element-subcycles per second (elements x subcycles x steps / time)
  roofline      the dominant kernel (the subcycle kernel of the tuned launch
                configuration) against the HBM roofline: its algorithmic bytes
                per launch (per-subcycle bytes x subcycles per launch) over its
                average launch duration, i.e. the HIP-event time of the timed
                region on the context's stream minus the start-of-step kernels
                and any remainder launch, divided by the number of launches;
                traffic = measured HBM bytes per launch from profiles/traffic.json
                when recorded for the current kernel sources
  cpu_baseline  the FP64 oracle on the host cores, on a bounded sample
  cpu_baseline_1thread  the same oracle on one host thread (one time step)
  advection     the DG advection of H and A (three Runge-Kutta stages), timed
                outside the region: ms per step, algorithmic bytes, GB/s
  variants      the same measurement for mixed precision, other launch
                strategies, the larger meshes, the 64-domain batch, general and
                curved cells and n_s = 8

The default workload is the largest single-domain one: 2048 x 2048 cells
(0.25 km on a 512 km square, 4.2M elements, 16.8M CG2 nodes, ~3 GB of state),
6 DG stress dofs, FP64, 100 subcycles per step. Its state does not fit the
256 MB Infinity Cache, so every launch streams from HBM. Variants whose
working set does fit (256 x 256, 32 x 32) are labelled cache-resident and
report their bound as latency/issue rather than HBM.
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
FP64_PEAK_TFS = 78.6           # MI355X FP64 vector (and matrix) peak
MALL_BYTES = 256 << 20         # MI355X Infinity Cache (last-level, all XCDs)
# FP64 operations of the parallelogram-cell element and node update per
# element-subcycle at n_s = 6 (multiplies, adds and fused multiply-adds counted
# as one operation each, from the arithmetic as written; flops = ops + FMAs)
FP64_FLOP_PER_ELEMENT_SUBCYCLE = 1600.0
TRAFFIC_PATH = os.path.join(ROOT, "profiles", "traffic.json")  # measured bytes per launch
METRIC = "element-subcycles/sec (FP64 vs mixed/batched) + achieved HBM GB/s vs peak"
# every source file that holds device code, the build script with its
# compiler flags and the runtime that orders the tiles (the traffic records
# are tied to a hash of them)
KERNEL_SOURCES = ["paper_2402_00466_amd/csrc/mevp_api.hip",
                  "paper_2402_00466_amd/csrc/mevp_device.hpp",
                  "paper_2402_00466_amd/csrc/mevp_kernels.hip",
                  "paper_2402_00466_amd/csrc/mevp_kernels_ns3.hip",
                  "paper_2402_00466_amd/csrc/mevp_kernels_ns6.hip",
                  "paper_2402_00466_amd/csrc/mevp_kernels_ns8.hip",
                  "paper_2402_00466_amd/csrc/mevp_kernels_affine.hip",
                  "paper_2402_00466_amd/csrc/mevp_kernels_affine_ns6_fp64.hip",
                  "paper_2402_00466_amd/csrc/mevp_affine.hpp",
                  "paper_2402_00466_amd/build.py",
                  "paper_2402_00466_amd/csrc/mevp_ref.hpp",
                  "paper_2402_00466_amd/csrc/mevp_internal.hpp",
                  "paper_2402_00466_amd/csrc/mevp_index.hpp",
                  "paper_2402_00466_amd/csrc/mevp_kernels_bf16.hip"]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def alg_bytes(domains, precision):
    """Algorithmic HBM bytes of one subcycle (what the method must move if
    nothing stays on chip between subcycles), per the definition used
    throughout: per element S read + write (2 x 3 n_s words of w_S bytes) and
    H, A (2 n_a doubles); 16 B per vertex (on-the-fly geometry); per CG2 node
    v read + write (32 B) and 8 doubles of per-step node data (v^n, ocean,
    air stress, M^H, m^A: 64 B). Element forces, tiles' halo re-reads and the
    like are implementation traffic and not counted.
    Returns (subcycle bytes, element-phase share, node-phase share); the two
    shares split the subcycle for the two-phase launch strategy (the element
    phase also reads v: 16 B per node)."""
    ws = 8 if precision == "fp64" else 4
    tot = be = bn = 0
    for d in domains:
        ne, nn, nv = d.nx * d.ny, (2 * d.nx + 1) * (2 * d.ny + 1), (d.nx + 1) * (d.ny + 1)
        per_e = ne * (2 * 3 * d.n_s * ws + 2 * d.n_a * 8) + nv * 16
        tot += per_e + nn * 96
        be += per_e + nn * 16
        bn += nn * 96
    return tot, be, bn


def advect_bytes(domains):
    """Algorithmic HBM bytes of one advection step of H and A (three SSP
    Runge-Kutta stages, each a pass over the elements): per stage the stage's
    input coefficients (2 n_a doubles per element) and, after the first stage,
    the step's start values as well, the output coefficients, the CG2 velocity
    (16 B per node) and the geometry (16 B per vertex). Neighbours' traces are
    the same coefficients again and not counted twice."""
    tot = 0
    for d in domains:
        ne, nn, nv = d.nx * d.ny, (2 * d.nx + 1) * (2 * d.ny + 1), (d.nx + 1) * (d.ny + 1)
        u = ne * 2 * d.n_a * 8
        for stage in range(3):
            tot += u * (1 if stage == 0 else 2) + u + nn * 16 + nv * 16
    return tot


def load_traffic(workload, precision, strategy, tile):
    """HBM traffic per launch of the dominant kernel from committed rocprofv3
    PMC summaries, if they were taken on the current kernel sources; else None."""
    path = TRAFFIC_PATH
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(f"{workload}/{precision}/{strategy}/{tile[0]}x{tile[1]}")
    except (ValueError, OSError):
        return None
    if not rec or rec.get("kernel_hash") != kernel_hash():
        return None
    return rec.get("bytes_per_launch")


def run_gpu(domains, precision, steps, warmup, n_sub, strategy=None, tile=None, tune=True):
    """Upload, optionally autotune (outside the timed region), warm up, then time
    ``steps`` steps with one event pair around them. Returns the timings and the
    launch configuration used."""
    import torch
    import paper_2402_00466_amd as M
    ctx = M.Context([M.Domain(d.nx, d.ny, d.n_s, d.n_a) for d in domains], precision=precision)
    for k, d in enumerate(domains):
        ctx.upload(k, d)
    ctx.check_inputs()
    # let the GPU clocks settle before tuning and again before timing: a short
    # workload otherwise runs its first milliseconds at lower clocks, and the
    # tuner's host round trips of the state let them drop (measured: the first
    # 10 steps after tuning ran ~5 % slow at 256 x 256). ~0.3 s of steps each;
    # the state they leave is the warm-up's starting point.
    def settle():
        t_settle = time.perf_counter()
        while True:
            ctx.step(n_sub)
            ctx.sync()
            if time.perf_counter() - t_settle > 0.3:
                break
    settle()
    if strategy is None and tune:
        ctx.tune(n_trial=max(10, min(n_sub, 50)))
    elif strategy is not None:
        ctx.set_config(strategy, tile or (16, 14))
    config = ctx.get_config()
    depth = ctx.launch_depth()  # subcycles per launch after the cell-kind fallbacks
    settle()
    for _ in range(warmup):
        ctx.step(n_sub)
    # start-of-step kernel alone (subtracted from the region to get the subcycle kernels)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ctx.sync()
    ev[0].record(ctx.stream)
    for _ in range(3):
        ctx.begin_step()
    ev[1].record(ctx.stream)
    torch.cuda.synchronize()
    begin_ms = ev[0].elapsed_time(ev[1]) / 3
    # the launch that ends a step when the subcycles per launch do not divide
    # n_sub (subtracted too, so the average is that of the dominant kernel alone)
    rem = n_sub % depth if depth > 1 else 0
    rem_ms = 0.0
    if rem:
        ev[0].record(ctx.stream)
        for _ in range(3):
            ctx.subcycles(rem)
        ev[1].record(ctx.stream)
        torch.cuda.synchronize()
        rem_ms = ev[0].elapsed_time(ev[1]) / 3
    # the timed region: `steps` whole steps, events only at its ends
    t0 = time.perf_counter()
    ev[2].record(ctx.stream)
    for _ in range(steps):
        ctx.step(n_sub)
    ev[3].record(ctx.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev[2].elapsed_time(ev[3])
    ctx.check_state()
    # advection of H and A (once per step before the subcycles; outside the timed region)
    ev[0].record(ctx.stream)
    for _ in range(3):
        ctx.advect()
    ev[1].record(ctx.stream)
    torch.cuda.synchronize()
    advect_ms = ev[0].elapsed_time(ev[1]) / 3
    # diagnostics outside the timed region: per-launch events over one step
    ctx.timing_enable(n_sub + 8)
    ctx.step(n_sub)
    tim = ctx.timing_read()
    ctx.timing_enable(0)
    ctx.close()
    del ctx
    torch.cuda.synchronize()
    return ms, wall, begin_ms, rem_ms, tim, config, advect_ms, depth


def measure(domains, precision, steps, warmup, n_sub, workload, strategy=None, tile=None):
    ms, wall, begin_ms, rem_ms, tim, config, advect_ms, depth = run_gpu(
        domains, precision, steps, warmup, n_sub, strategy, tile)
    strategy, tile = config
    el_sub = sum(d.nx * d.ny for d in domains) * n_sub * steps
    value = el_sub / (ms * 1e-3)
    tot, be, bn = alg_bytes(domains, precision)
    # launches of the subcycle kernel(s) in the timed region
    # (depth: what the library runs per launch for this configuration and these
    # cells, e.g. one subcycle for fused_pair with curved cells)
    if depth == 0:
        launches, per_launch, kernel = steps, n_sub, "k_fused_persist (all subcycles of a step)"
    elif strategy == "two_phase":
        launches, per_launch, kernel = steps * n_sub, 1, "k_element + k_node (two-phase subcycle)"
    elif depth > 1:
        launches, per_launch = steps * (n_sub // depth), depth
        kernel = f"k_fused_multi (K = {depth} subcycles per launch)"
    else:
        launches, per_launch, kernel = steps * n_sub, 1, "k_fused (one subcycle)"
    # average launch duration of the dominant kernel: the timed region minus the
    # start-of-step kernel and any remainder launch of each step
    kms = max(ms - steps * (begin_ms + rem_ms), 1e-9) / max(launches, 1)
    kbytes = tot * per_launch
    # advection of H and A, timed outside the region (one call = one step)
    ab = advect_bytes(domains)
    ab_gbs = ab / (max(advect_ms, 1e-9) * 1e-3) / 1e9
    c0, t0 = tim["element"]
    c1, t1 = tim["node"]
    return {
        "value": value, "ms_per_step": ms / steps, "wall_s": wall,
        "config": {"strategy": strategy, "tile": list(tile)},
        "kernels_ms": {"dominant_avg": kms, "begin_step": begin_ms, "remainder_launch": rem_ms,
                       "advect_step": advect_ms,
                       "diag_per_launch_events": {"subcycle_or_element_avg": t0 / max(c0, 1),
                                                  "node_avg": t1 / c1 if c1 else None,
                                                  "launches": c0}},
        "advection": {"kernel": "k_advect (3 stages per step)", "ms_per_step": advect_ms,
                      "alg_bytes_per_step": ab, "achieved_GBs": ab_gbs,
                      "frac": ab_gbs / HBM_PEAK_GBS},
        "roofline": roofline(domains, precision, workload, strategy, tile, kernel, kbytes,
                             kms, per_launch),
    }


def roofline(domains, precision, workload, strategy, tile, kernel, kbytes, kms, per_launch):
    """The dominant kernel against the HBM roofline. ``achieved`` is the
    method's algorithmic bytes per launch over the launch's average duration
    (the rate of a program that streams exactly the method's bytes). Beside
    it: the bytes the kernel really moves (rocprofv3 FETCH_SIZE + WRITE_SIZE,
    when recorded for the current sources) over the same time, and its useful
    FP64 arithmetic rate against the FP64 peak. A working set that fits the
    Infinity Cache is not bound by HBM: such workloads say so."""
    achieved = kbytes / (kms * 1e-3) / 1e9
    traffic = load_traffic(workload, precision, strategy, tile)
    ws = working_set_bytes(domains, precision)
    resident = ws <= MALL_BYTES
    elems = sum(d.nx * d.ny for d in domains)
    r = {"bound": "latency/issue (cache-resident)" if resident else "hbm",
         "kernel": kernel, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
         "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
         "alg_bytes_per_launch": kbytes, "subcycles_per_launch": per_launch,
         "working_set_bytes": ws, "achieved_is": "algorithmic bytes per launch / launch time"}
    if traffic:
        r["measured_GBs"] = traffic / (kms * 1e-3) / 1e9
        r["measured_frac"] = r["measured_GBs"] / HBM_PEAK_GBS
    if precision == "fp64" and workload.endswith("-dg2") and not workload.startswith("batch"):
        tfs = FP64_FLOP_PER_ELEMENT_SUBCYCLE * elems * per_launch / (kms * 1e-3) / 1e12
        r["fp64_TFs"] = tfs
        r["fp64_frac"] = tfs / FP64_PEAK_TFS
    return r


def traffic_probe(workload, precision, strategy, tile, n_sub, copy_mib):
    """A short run for hardware-counter collection (rocprofv3 --pmc): a device
    copy of ``copy_mib`` MiB (reads and writes exactly that many bytes; the
    calibration of the byte counters), then one start-of-step kernel and
    ``n_sub`` subcycles of the workload."""
    import torch
    from synth_inputs import named_workload
    import paper_2402_00466_amd as M
    n = copy_mib * (1 << 20) // 8
    src = torch.arange(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    doms = named_workload(workload)
    ctx = M.Context([M.Domain(d.nx, d.ny, d.n_s, d.n_a) for d in doms], precision=precision)
    ctx.set_config(strategy, tile)
    ctx.set_graph(False)
    for k, d in enumerate(doms):
        ctx.upload(k, d)
    ctx.step(n_sub)
    ctx.sync()
    log(f"probe done: copy {copy_mib} MiB x2, {workload} {precision} {strategy} {tile} "
        f"{n_sub} subcycles")


def record_traffic(key, fetch_csv, write_csv, copy_mib, kernel_substr, command):
    """Turn the two rocprofv3 PMC runs of the probe into a traffic record:
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the dominant kernel, each
    scaled by the factor that makes the same counter read exactly ``copy_mib``
    MiB for the probe's device copy. Stored in profiles/traffic.json under
    ``key`` with the current kernel-source hash."""
    import csv

    def rows(path):
        return list(csv.DictReader(open(path)))

    out = {}
    for name, path in (("fetch", fetch_csv), ("write", write_csv)):
        r = rows(path)
        copies = sorted((float(x["Counter_Value"]) for x in r if "copyBuffer" in x["Kernel_Name"]),
                        reverse=True)[:2]  # the two copies of copy_mib MiB are the largest
        kern = [float(x["Counter_Value"]) for x in r if kernel_substr in x["Kernel_Name"]]
        if len(copies) < 2 or not kern:
            raise SystemExit(f"{path}: probe copies or kernel {kernel_substr!r} not found")
        factor = copy_mib * 1024.0 / (sum(copies) / len(copies))
        out[name] = {"kib_per_dispatch": sum(kern) / len(kern), "dispatches": len(kern),
                     "copy_kib": sum(copies) / len(copies), "scale": factor}
    total = (out["fetch"]["kib_per_dispatch"] * out["fetch"]["scale"] +
             out["write"]["kib_per_dispatch"] * out["write"]["scale"]) * 1024.0
    path = TRAFFIC_PATH
    db = json.load(open(path)) if os.path.exists(path) else {}
    db[key] = {"bytes_per_launch": total, "fetch": out["fetch"], "write": out["write"],
               "kernel": kernel_substr, "kernel_hash": kernel_hash(), "command": command}
    json.dump(db, open(path, "w"), indent=1, sort_keys=True)
    print(json.dumps({key: db[key]}))


def oracle_mesh(d):
    import oracle
    return oracle.Mesh(d.nx, d.ny, d.n_s, d.n_a, d.vertices)


def cpu_baseline(domains, n_sub, budget_s, chunk, m=None):
    """The FP64 oracle as it stands, on the host, on a bounded sample of the
    workload: the first domain, whole mesh, advanced from rest in calls of
    ``chunk`` subcycles (each call a time step of that many subcycles: the
    start-of-step work once, then the subcycles) until ``budget_s`` of wall
    time is spent (at least one call, at most ``n_sub`` x 40 subcycles)."""
    import oracle
    d = domains[0]
    m = m or oracle_mesh(d)
    p = oracle.Params()
    v = S = None
    done = 0
    t0 = time.perf_counter()
    while True:
        v, S = m.run(p, d.H, d.A, d.wind, d.ocean, 1, chunk, v=v, S=S)
        done += chunk
        el = time.perf_counter() - t0
        if el >= budget_s or done >= 40 * n_sub:
            break
    return {"value": d.nx * d.ny * done / el, "unit": "element-subcycles/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{done // chunk} call(s) x {chunk} subcycles on the whole {d.nx}x{d.ny} "
                      f"mesh (n_s={d.n_s}) from rest, {el:.1f} s"}


def cpu_baseline_1thread(domains, n_sub, chunk, m=None):
    """The same oracle on one host thread: one call of ``chunk`` subcycles."""
    import oracle
    threads = oracle.num_threads()
    oracle.set_num_threads(1)
    try:
        r = cpu_baseline(domains, n_sub, 0.0, chunk, m)
    finally:
        oracle.set_num_threads(threads)
    return r


def working_set_bytes(domains, precision):
    """Device bytes the subcycle kernels touch (the context's workspace)."""
    import paper_2402_00466_amd as M
    return M.workspace_size([M.Domain(d.nx, d.ny, d.n_s, d.n_a) for d in domains], precision)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n-sub", type=int, default=100)
    ap.add_argument("--workload", default="2048x2048-dg2")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed", "mixed_bf16"])
    ap.add_argument("--strategy", default=None,
                    choices=["fused", "two_phase", "persistent", "fused_pair", "fused_triple"],
                    help="launch strategy; default: autotuned (mevp_tune) before the timed region")
    ap.add_argument("--tile", default=None, help="owned tile, e.g. 16x14 (with --strategy)")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=12.0)
    ap.add_argument("--cpu-chunk", type=int, default=10,
                    help="subcycles per oracle call in the CPU baseline (a bounded sample)")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="only run the short counter-collection probe (see traffic_probe)")
    ap.add_argument("--copy-mib", type=int, default=1024)
    ap.add_argument("--record-traffic", nargs=3, metavar=("KEY", "FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/traffic.json[KEY] from the probe's two PMC runs")
    ap.add_argument("--record-command", default="", help="command line stored with the record")
    args = ap.parse_args()
    if args.record_traffic:
        key, fcsv, wcsv = args.record_traffic
        strategy = key.split("/")[2]
        kern = {"two_phase": "k_element<", "fused_pair": "k_fused_multi<",
                "fused_triple": "k_fused_multi<"}.get(strategy, "k_fused<")
        record_traffic(key, fcsv, wcsv, args.copy_mib, kern, args.record_command)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}): the mEVP subcycle "
              "here runs on a single GPU; a multi-GPU decomposition is not built", file=sys.stderr)
        sys.exit(2)

    import torch
    from synth_inputs import named_workload
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    torch.cuda.set_device(0)
    import paper_2402_00466_amd as M
    M.lib()
    tile = tuple(int(x) for x in args.tile.split("x")) if args.tile else None
    if args.traffic_probe:
        strategy = args.strategy or "fused"
        # whole launches of the kernel only
        n_probe = {"fused_pair": 4, "fused_triple": 6}.get(strategy, 3)
        traffic_probe(args.workload, args.precision, strategy, tile or (16, 14),
                      args.n_sub if args.n_sub != 100 else n_probe, args.copy_mib)
        return

    log(f"workload {args.workload} {args.precision}: generating inputs")
    doms = named_workload(args.workload)
    head = measure(doms, args.precision, args.steps, args.warmup, args.n_sub, args.workload,
                   args.strategy, tile)
    log(f"headline {head['value']:.3e} element-subcycles/s, {head['ms_per_step']:.3f} ms/step, "
        f"{head['config']}, {head['roofline']['frac']:.3f} of HBM peak")

    variants = {}
    if not args.no_variants:
        other = "mixed" if args.precision == "fp64" else "fp64"
        plan = [(args.workload, other, args.steps, None, None),
                (args.workload, args.precision, 3, "two_phase", None),
                (args.workload, args.precision, 3, "fused", (16, 14)),
                (args.workload, args.precision, 3, "fused_pair", (13, 13)),
                ("256x256-dg2", "fp64", 10, None, None), ("256x256-dg2", "mixed", 10, None, None),
                ("256x256-dg2", "fp64", 10, "two_phase", None),
                ("256x256-dg2", "fp64", 10, "fused", (16, 16)),
                ("256x256-dg2", "fp64", 3, "persistent", (16, 16)),
                ("1024x1024-dg2", "fp64", 3, None, None), ("1024x1024-dg2", "mixed", 3, None, None),
                ("batch64-dg2", "fp64", 2, None, None), ("batch64-dg2", "mixed", 2, None, None),
                ("2048x2048-dg2-bilinear", "fp64", 2, None, None),
                ("2048x2048-dg2-bilinear", "mixed", 2, None, None),
                ("2048x2048-dg2", "mixed_bf16", 3, None, None),
                ("2048x2048-dg2-bilinear", "mixed_bf16", 2, None, None),
                ("1024x1024-ns8", "fp64", 2, None, None), ("1024x1024-ns8", "mixed", 2, None, None),
                ("1024x1024-dg2-iso", "fp64", 2, None, None),
                ("1024x1024-dg2-iso", "mixed", 2, None, None),
                ("32x32-dg1", "fp64", 10, None, None), ("32x32-dg1", "mixed", 10, None, None)]
        plan = [x for x in plan if (x[0], x[1], x[3], x[4]) != (args.workload, args.precision,
                                                                 None, None)]
        for wl, prec, st, strat, tl in plan:
            log(f"variant {wl} {prec} {strat or 'tuned'} {tl or ''} ({st} steps)")
            ds = doms if wl == args.workload else named_workload(wl)
            r = measure(ds, prec, st, 1, args.n_sub, wl, strat, tl)
            key = f"{wl}/{prec}/" + (f"{strat}/{tl[0]}x{tl[1]}" if strat and tl else (strat or "tuned"))
            variants[key] = {
                "value": r["value"], "ms_per_step": r["ms_per_step"], "steps": st,
                "elements": sum(d.nx * d.ny for d in ds), "config": r["config"],
                "dominant_kernel_ms": r["kernels_ms"]["dominant_avg"],
                "bound": r["roofline"]["bound"],
                "roofline_frac": r["roofline"]["frac"],
                "achieved_GBs": r["roofline"]["achieved"],
                "advection_frac": r["advection"]["frac"]}
            if r["roofline"].get("measured_GBs"):
                variants[key]["measured_GBs"] = r["roofline"]["measured_GBs"]
                variants[key]["measured_frac"] = r["roofline"]["measured_frac"]
            log(f"  {r['value']:.3e} element-subcycles/s ({r['config']['strategy']} "
                f"{r['config']['tile']}), {r['roofline']['frac']:.3f} of HBM peak")
            del ds
        # the persistent kernel's grid-wide barrier: its per-step kernel time
        # against the single-subcycle kernel's (same tiles, one tile per
        # workgroup at 256 x 256) over the 99 barriers of a 100-subcycle step
        per = variants.get("256x256-dg2/fp64/persistent/16x16")
        one = variants.get("256x256-dg2/fp64/fused/16x16")
        if per and one and args.n_sub > 1:
            variants["persistent_barrier_us"] = 1e3 * (
                per["dominant_kernel_ms"] - args.n_sub * one["dominant_kernel_ms"]) / (args.n_sub - 1)
        mix = variants.get(f"{args.workload}/mixed/tuned")
        if mix and args.precision == "fp64" and args.strategy is None:
            variants["mixed_speedup_over_fp64"] = mix["value"] / head["value"]
        for wl in ("256x256-dg2", "1024x1024-dg2", "batch64-dg2", "2048x2048-dg2-bilinear",
                   "1024x1024-ns8", "1024x1024-dg2-iso", "32x32-dg1"):
            a, b = variants.get(f"{wl}/mixed/tuned"), variants.get(f"{wl}/fp64/tuned")
            if a and b:
                variants[f"{wl}/mixed_speedup_over_fp64"] = a["value"] / b["value"]
        # the bfloat16 element-matrix trial against the mixed form and FP64
        for wl in (args.workload, "2048x2048-dg2-bilinear"):
            bf = variants.get(f"{wl}/mixed_bf16/tuned")
            mx = variants.get(f"{wl}/mixed/tuned")
            f64 = variants.get(f"{wl}/fp64/tuned") or (head if wl == args.workload and
                                                        args.precision == "fp64" else None)
            if bf and mx:
                variants[f"{wl}/mixed_bf16_speedup_over_mixed"] = bf["value"] / mx["value"]
            if bf and f64:
                variants[f"{wl}/mixed_bf16_speedup_over_fp64"] = bf["value"] / f64["value"]

    cpu = cpu1 = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        m = oracle_mesh(doms[0])
        cpu = cpu_baseline(doms, args.n_sub, args.cpu_budget, args.cpu_chunk, m)
        cpu1 = cpu_baseline_1thread(doms, args.n_sub, max(1, args.cpu_chunk // 5), m)
        del m

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
        "dtype": {"fp64": "f64", "mixed": "f32+f64", "mixed_bf16": "bf16 matrices+f32+f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": args.workload, "precision": args.precision,
                   "strategy": head["config"]["strategy"], "tile": head["config"]["tile"],
                   "domains": len(doms), "elements": sum(d.nx * d.ny for d in doms),
                   "mesh": f"{d0.nx}x{d0.ny}", "n_s": d0.n_s, "n_a": d0.n_a,
                   "n_sub": args.n_sub, "step": "one mEVP time step (start-of-step kernel + n_sub subcycles)"},
        "roofline": head["roofline"],
        "kernels_ms": head["kernels_ms"],
        "advection": head["advection"],
        "cpu_baseline": cpu,
        "cpu_baseline_1thread": cpu1,
        "variants": variants,
        "kernel_hash": kernel_hash(),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
