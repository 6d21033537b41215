"""Host logic of bench.py (no GPU): the one-GPU guard, the algorithmic byte
count, the counter and trace summaries on synthetic rocprofv3 CSV files, and
the lookup of the committed traffic figure by kernel sources and knobs."""
import csv
import importlib.util
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_section_child_failure_is_reported_not_raised(bench):
    """A section run in a child process that fails comes back as an error
    entry (here: the child refuses a second GPU before touching any)."""
    r = bench.run_section_child("serve", None, ["--gpus", "2"])
    assert r == {"error": "section serve exited with status 2"}


def test_serving_flags_are_accepted_by_the_child(bench):
    import argparse
    args = argparse.Namespace(d=0.85, serve_rate=2000.0, serve_seconds=5.0,
                              serve_sustained_seconds=60.0, serve_warmup=1.0, serve_burst=2000,
                              serve_solo=100, serve_hbm_gib=32, no_autotune=True)
    f = bench.serve_forward(args)
    assert "--no-autotune" in f
    # parsed by the child's own argument parser (then refused at the GPU guard)
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--section", "serve",
                        "--gpus", "2"] + f, capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "exactly one GPU" in r.stderr


def test_algorithmic_bytes(bench):
    st = {"rounds": 3, "nodes_diffused": 10, "edges_diffused": 100}
    # fp32: 4 B per node scanned per round, 52 B per taken node, 12 B per link
    assert bench.algorithmic_bytes(1000, st, "fp32") == 4 * 1000 * 3 + 52 * 10 + 12 * 100
    assert bench.algorithmic_bytes(1000, st, "fp64") == 8 * 1000 * 3 + 64 * 10 + 20 * 100


def _counter_csv(path, counter, rows):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name",
                                           "Counter_Value"])
        w.writeheader()
        for i, (name, v) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": name, "Counter_Name": counter,
                        "Counter_Value": v})


def test_summarize_counters_scales_by_the_copy(bench, tmp_path):
    copy_kib = 1024 * 1024  # a 1 GiB copy
    kr = "void di::k_round<float, 1, 512>(di::DiArgs<float>, int, int)"
    fetch = tmp_path / "fetch.csv"
    write = tmp_path / "write.csv"
    # two working dispatches and one launch after the stop, which loads its
    # inputs (a large FETCH) but writes nothing: the write run excludes it from both
    _counter_csv(fetch, "FETCH_SIZE", [(kr, 1000.0), (kr, 3000.0), (kr, 900.0),
                                       ("__amd_rocclr_copyBuffer", copy_kib * 0.5)])
    _counter_csv(write, "WRITE_SIZE", [(kr, 500.0), (kr, 700.0), (kr, 0.0),
                                       ("__amd_rocclr_copyBuffer", copy_kib * 1.0)])
    out = tmp_path / "traffic.json"
    knobs = ["op2", 0.03125, 11, 512]
    e = bench.summarize_counters(str(fetch), str(write), knobs, out_path=str(out))
    assert e["fetch_kib_per_dispatch"] == pytest.approx(2000.0 / 0.5)
    assert e["write_kib_per_dispatch"] == pytest.approx(600.0)
    assert e["raw"]["dispatches"] == [2, 2]
    t = json.loads(out.read_text())
    assert t["kernel_hash"] == bench.kernel_hash()
    # a second knob setting is added beside the first, the same one replaced
    bench.summarize_counters(str(fetch), str(write), ["op", 0.0625, 11, 512],
                             out_path=str(out))
    bench.summarize_counters(str(fetch), str(write), knobs, out_path=str(out))
    t = json.loads(out.read_text())
    assert sorted(x["knobs"][0] for x in t["entries"]) == ["op", "op2"]
    tune = {"schedule": "op2", "c": 0.03125, "window_log2": 11, "threads": 0}
    assert bench.measured_traffic(tune, path=str(out)) == pytest.approx((4000.0 + 600.0) * 1024)
    assert bench.measured_traffic(dict(tune, c=0.0625), path=str(out)) is None
    # counters taken on other kernel sources are not reported
    t["kernel_hash"] = "0" * 16
    out.write_text(json.dumps(t))
    assert bench.measured_traffic(tune, path=str(out)) is None


def test_committed_traffic_only_reported_for_its_kernel_sources(bench):
    """The committed counter summary is reported (bytes > 0 at each knob setting
    it holds) while the kernel sources still hash to the value it records;
    once they have changed, bench.py reports no traffic (None) instead of
    figures taken on other code."""
    with open(bench.TRAFFIC_FILE) as fh:
        raw = json.load(fh)
    current = raw.get("kernel_hash") == bench.kernel_hash()
    assert bool(bench.load_traffic()) == current
    for e in raw["entries"]:
        sc, c, wlog, threads = e["knobs"]
        tune = {"schedule": sc, "c": c, "window_log2": wlog, "threads": threads}
        if current:
            assert bench.measured_traffic(tune) > 0
        else:
            assert bench.measured_traffic(tune) is None


def test_summarize_trace_separates_launches_after_the_stop(bench, tmp_path, capsys):
    path = tmp_path / "trace.csv"
    kr = "void di::k_round<float, 0, 512>(di::DiArgs<float>, int, int)"
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for dur_ns in (40000, 50000, 4000):
            w.writerow({"Kernel_Name": kr, "Start_Timestamp": 0, "End_Timestamp": dur_ns})
    bench.summarize_trace(str(path))
    line = capsys.readouterr().out.strip()
    assert "calls     3" in line and "working     2" in line
    assert "avg_working_us     45.00" in line and "returned-at-once 1" in line


def test_cpu_leg_times_the_oracle_and_returns_its_references(bench):
    """The CPU leg on a small graph: the sequential and OpenMP baselines are
    reported with their core counts, and each reference is the oracle's exact
    limit (direct solve for small graphs, MAT-ITER on every core otherwise)."""
    import numpy as np
    import oracle
    import workloads as wl
    g = wl.random_small(300, 1500, seed=3)
    big = wl.recipe("pagerank-10k", n=30000, seed=9)
    out, refs = bench.cpu_baseline(g, 0.85, 1e-8, 0.05,
                                   refs=[("small", g, 0.85, 0.0, None),
                                         ("big", big, 0.9, 1e-12, None)])
    assert out["cores"] == 1 and out["value"] > 0
    assert out["mat_iter_openmp"]["cores"] >= 1 and out["mat_iter_openmp"]["products"] > 0
    assert out["host"]["nproc"] >= 1
    assert set(refs) == {"small", "big"}
    assert np.abs(refs["small"] - oracle.dense_exact(g, 0.85)[1]).sum() < 1e-12
    # the sequential MAT-ITER (exact up to its own stop) on the larger graph
    seq = oracle.power(big, 0.9, 1e-13)["x"]
    assert np.abs(refs["big"] - seq).sum() < 2 * 0.9 * 1e-12 / 0.1 + 1e-12


def test_c1_knob_string(bench):
    assert bench.parse_c1_tune("op:0.03125:8:persist") == ("op", 0.03125, 8, True)
    assert bench.parse_c1_tune("op2:0.0625:9") == ("op2", 0.0625, 9, False)
    for bad in ["op:0.03125", "op:0.03125:8:persis", "max:1:8", "op:1:8:persist:x"]:
        with pytest.raises(SystemExit):
            bench.parse_c1_tune(bad)
