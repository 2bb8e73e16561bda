"""CPU checks of the benchmark script's contract parts that need no GPU: one
GPU only, the algorithmic-byte model, and the traffic record built from two
rocprofv3 PMC CSV files (scaled by the probe's device copy)."""
import csv
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_per_element_subcycle():
    """The per-unit byte model: 704.2 B per element-subcycle at 2048^2
    FP64 n_s = 6 (S 288 B, H+A 16 B, vertices 16 B, nodes 96 B each), 560.2 B
    mixed; 2.954 GB per subcycle."""
    import bench
    from synth_inputs import make_domain
    d = make_domain(2048, 2048, 6, 1, seed=1)
    tot64 = bench.alg_bytes([d], "fp64")[0]
    totmx = bench.alg_bytes([d], "mixed")[0]
    assert tot64 == 2048 * 2048 * (288 + 16) + 2049 ** 2 * 16 + 4097 ** 2 * 96
    assert abs(tot64 / 2048 ** 2 - 704.2) < 0.1
    assert abs(totmx / 2048 ** 2 - 560.2) < 0.1


def _pmc_csv(path, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, val in rows:
            w.writerow({"Kernel_Name": name, "Counter_Name": "X", "Counter_Value": val})


def test_traffic_record_scales_by_the_copy_calibration(tmp_path, monkeypatch):
    import bench
    monkeypatch.setattr(bench, "TRAFFIC_PATH", str(tmp_path / "traffic.json"))
    kern = "void mevp::(anonymous namespace)::k_fused_multi<6, 1, double, double, 0, 17, 17, 3>(x)"
    # 1 GiB copies read as 512 MiB by FETCH_SIZE (factor 2) and 1 GiB by WRITE_SIZE
    _pmc_csv(tmp_path / "f.csv", [("__amd_rocclr_copyBuffer", 524288.0),
                                  ("__amd_rocclr_copyBuffer", 524288.0),
                                  ("__amd_rocclr_copyBuffer", 8.0), (kern, 1000.0), (kern, 1200.0)])
    _pmc_csv(tmp_path / "w.csv", [("__amd_rocclr_copyBuffer", 1048576.0),
                                  ("__amd_rocclr_copyBuffer", 1048576.0), (kern, 500.0),
                                  (kern, 500.0)])
    bench.record_traffic("w/fp64/fused_triple/16x16", str(tmp_path / "f.csv"),
                         str(tmp_path / "w.csv"), 1024, "k_fused_multi<", "cmd")
    rec = json.load(open(tmp_path / "traffic.json"))["w/fp64/fused_triple/16x16"]
    assert rec["fetch"]["scale"] == pytest.approx(2.0) and rec["write"]["scale"] == pytest.approx(1.0)
    assert rec["bytes_per_launch"] == pytest.approx((1100.0 * 2.0 + 500.0) * 1024.0)
    assert rec["kernel_hash"] == bench.kernel_hash()
    # a record is used only while the kernel sources are unchanged
    assert bench.load_traffic("w", "fp64", "fused_triple", (16, 16)) == rec["bytes_per_launch"]
    rec["kernel_hash"] = "stale"
    json.dump({"w/fp64/fused_triple/16x16": rec}, open(tmp_path / "traffic.json", "w"))
    assert bench.load_traffic("w", "fp64", "fused_triple", (16, 16)) is None


@pytest.mark.parametrize("strategy,depth,launches,per_launch,kernel", [
    ("fused_triple", 3, 33, 3, "k_fused_multi (K = 3"),
    ("fused_triple", 2, 50, 2, "k_fused_multi (K = 2"),   # a bilinear domain present
    ("fused_pair", 1, 100, 1, "k_fused (one subcycle)"),   # curved cells
    ("fused", 1, 100, 1, "k_fused (one subcycle)"),
    ("two_phase", 1, 100, 1, "k_element + k_node"),
    ("persistent", 0, 1, 100, "k_fused_persist"),
    ("persistent", 1, 100, 1, "k_fused (one subcycle)"),  # several cell kinds
])
def test_dominant_kernel_follows_the_reported_launch_depth(monkeypatch, strategy, depth,
                                                           launches, per_launch, kernel):
    """measure() counts the dominant kernel's launches from the subcycles per
    launch the library reports (mevp_get_launch_depth), not from the strategy's
    name: one step of 100 subcycles, 1 ms of timed region, no start-of-step or
    remainder time."""
    import bench
    from synth_inputs import make_domain
    d = make_domain(8, 8, 6, 1, seed=1)
    tim = {"element": (launches, 1.0), "node": (0, 0.0)}
    monkeypatch.setattr(bench, "run_gpu", lambda *a, **k: (
        1.0, 0.01, 0.0, 0.0, tim, (strategy, (16, 14)), 0.0, depth))
    r = bench.measure([d], "fp64", 1, 0, 100, "8x8", strategy, (16, 14))
    rf = r["roofline"]
    assert rf["kernel"].startswith(kernel)
    assert rf["subcycles_per_launch"] == per_launch
    assert r["kernels_ms"]["dominant_avg"] == pytest.approx(1.0 / launches)
    tot = bench.alg_bytes([d], "fp64")[0]
    # bytes per launch x launches / time: the method's bytes for the whole region
    assert rf["achieved"] * 1e9 * 1e-3 == pytest.approx(tot * per_launch * launches)


def test_advection_bytes_per_step():
    """Three stages: the first reads U^n, the others U^n and the stage input;
    each writes its output and reads the CG2 velocity and the vertices once."""
    import bench
    from synth_inputs import make_domain
    d = make_domain(8, 6, 6, 3, seed=1)
    u = 8 * 6 * 2 * 3 * 8
    per_stage_v_geo = 17 * 13 * 16 + 9 * 7 * 16
    assert bench.advect_bytes([d]) == (u + u) + 2 * (2 * u + u) + 3 * per_stage_v_geo


@pytest.mark.parametrize("ws,bound", [(5 << 30, "hbm"), (64 << 20, "latency/issue (cache-resident)")])
def test_roofline_fields_with_and_without_a_traffic_record(monkeypatch, ws, bound):
    """The roofline object: `achieved` is the algorithmic bytes per launch over
    the launch time; a traffic record for the current sources adds the measured
    HBM rate and fraction over the same time; a working set that fits the
    Infinity Cache is labelled cache-resident; the FP64 rate is reported for
    the single-domain DG2 FP64 workloads only."""
    import bench
    from synth_inputs import make_domain
    d = make_domain(8, 8, 6, 1, seed=1)
    monkeypatch.setattr(bench, "working_set_bytes", lambda *a: ws)
    kbytes, kms = 3.0e9, 0.5
    for traffic in (1.5e9, None):
        monkeypatch.setattr(bench, "load_traffic", lambda *a, t=traffic: t)
        r = bench.roofline([d], "fp64", "8x8-dg2", "fused_triple", (16, 16), "k", kbytes, kms, 3)
        assert r["bound"] == bound and r["unit"] == "GB/s" and r["peak"] == bench.HBM_PEAK_GBS
        assert r["achieved"] == pytest.approx(kbytes / 0.5e-3 / 1e9)
        assert r["frac"] == pytest.approx(r["achieved"] / bench.HBM_PEAK_GBS)
        assert r["traffic"] == traffic
        if traffic:
            assert r["measured_GBs"] == pytest.approx(traffic / 0.5e-3 / 1e9)
            assert r["measured_frac"] == pytest.approx(r["measured_GBs"] / bench.HBM_PEAK_GBS)
        else:
            assert "measured_GBs" not in r and "measured_frac" not in r
        assert r["fp64_TFs"] == pytest.approx(
            bench.FP64_FLOP_PER_ELEMENT_SUBCYCLE * 64 * 3 / 0.5e-3 / 1e12)
    r = bench.roofline([d], "mixed", "8x8-dg2", "fused_triple", (16, 16), "k", kbytes, kms, 3)
    assert "fp64_TFs" not in r
