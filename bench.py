#!/usr/bin/env python3
"""Benchmark: D-iteration PageRank on one MI355X (gfx950).

One step = one D-iteration solve of the workload graph (uniform V, d = 0.85)
from F_0 = (1-d)V to ||F||_1 < tol, with the result normalised, inputs already
resident in HBM.  Prints ONE JSON line with:

  value           solves per second (whole job, one GPU)
  roofline        the round kernel: algorithmic bytes per launch (4 B per node
                  scanned, 52 B per node taken, 12 B per link pushed for fp32
                  fluid; 8 / 64 / 20 B for fp64) over its average launch
                  duration, timed with HIP events on the solve's stream
  comparator      the GPU power iteration (pull) on the same graph and stop rule
  cpu_baseline    the CPU oracle's sequential D-iteration on the host
  ppr_batch       batched personalised PageRank (256 seed sets, 1e-6)
  update          a 1% graph change: injected fluid + resume vs a fresh solve
  paper_replay    the paper's six simulation scenarios: links diffused vs power iteration
  serve           the continuous-batching server on a short Poisson stream

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
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

METRIC = ("time to L1 residual 1e-8 & edges diffused/s vs GPU power iter; "
          "PPR queries/s, p50/p99")
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "round_kernel_traffic.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1202_6158_amd", "csrc", f)
                  for f in ("diter.hip", "kernels.h", "internal.h")]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def algorithmic_bytes(n, st, precision):
    """Bytes the D-iteration must move for one solve (scan of F per round,
    per taken node, per pushed link), excluding the final flush."""
    if precision == "fp64":
        return 8 * n * st["rounds"] + 64 * st["nodes_diffused"] + 20 * st["edges_diffused"]
    return 4 * n * st["rounds"] + 52 * st["nodes_diffused"] + 12 * st["edges_diffused"]


def launch_knobs(tune):
    """(schedule, c, window_log2, threads) of a tune dict, threads 0 read as
    the library's default of 512."""
    if not tune:
        return None
    return [tune["schedule"], round(float(tune["c"]), 6), int(tune["window_log2"]),
            int(tune["threads"]) or 512]


def load_traffic(path=TRAFFIC_FILE):
    """The counter summary, or {} when absent or taken on other kernel sources."""
    try:
        with open(path) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return {}
    return t if t.get("kernel_hash") == kernel_hash() else {}


def measured_traffic(tune, path=TRAFFIC_FILE):
    """HBM bytes per round-kernel launch from the committed counter summary,
    or None when absent, taken on other kernel sources or not taken at these
    knobs (the knobs set the work of a launch)."""
    for e in load_traffic(path).get("entries", []):
        if e["knobs"] == launch_knobs(tune):
            return (e["fetch_kib_per_dispatch"] + e["write_kib_per_dispatch"]) * 1024.0
    return None


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(g, d, tol, budget_s, refs=()):
    """The CPU leg: the oracle timed on the host, and the oracle's references.

    - value: the oracle's sequential D-iteration (threshold sweeps, fp64, one
      thread) on the benchmark graph, full solves to ||F||_1 < tol.
    - mat_iter_openmp: the oracle's MAT-ITER on every host core to the same
      stop rule, on the same graph.
    - references: for each (name, graph, d, ref_tol, v) in refs, the oracle's
      limit (MAT-ITER on every core until ||X_n - X_n-1||_1 < ref_tol, or a
      sparse direct solve up to 2e4 nodes), normalised; returned apart (as
      numpy vectors) for the L1 errors of the GPU results.
    Returns (summary dict, {name: x_ref})."""
    import oracle
    oracle.build(force=False)
    runs, t0 = 0, time.perf_counter()
    while True:
        r = oracle.diter(g, d, tol, order="sweep", c=1.0)
        runs += 1
        el = time.perf_counter() - t0
        if el >= budget_s or runs >= 100:
            break
    out = {"value": runs / el, "unit": "solves/s", "cores": 1, "kind": "oracle",
           "sample": "%d full solve(s) of the benchmark graph to ||F||_1 < %g by the oracle's "
                     "sequential threshold-sweep D-iteration (fp64, one thread), %.1f s" %
                     (runs, tol, el),
           "edges_per_s": r["stats"]["edges"] / (el / runs),
           "host": {"nproc": os.cpu_count(), "cpu_model": cpu_model()}}
    t0 = time.perf_counter()
    p = oracle.power_omp(g, d, tol)
    tp = time.perf_counter() - t0
    out["mat_iter_openmp"] = {"solves_per_s": 1.0 / tp, "seconds": tp, "cores": p["threads"],
                              "products": p["stats"]["rounds"],
                              "note": "the oracle's MAT-ITER (fp64 pull, OpenMP over rows) to "
                                      "||X_n - X_n-1||_1 < %g on every host core" % tol}
    ref_x, ref_info = {}, {}
    for name, rg, rd, rtol, rv in refs:
        t0 = time.perf_counter()
        if rg.n <= 20000:
            ref_x[name] = oracle.sparse_exact(rg, rd, v=rv)[1]
            how = "sparse direct solve of (I - dP) Y = (1-d) V"
        else:
            q = oracle.power_omp(rg, rd, rtol, v=rv)
            ref_x[name] = q["x"]
            how = ("MAT-ITER on %d cores to ||X_n - X_n-1||_1 < %g (%d products; its own L1 "
                   "bound %.1e)" % (q["threads"], rtol, q["stats"]["rounds"],
                                    2 * rd * q["stats"]["residual"] / (1 - rd)))
        ref_info[name] = {"how": how, "seconds": time.perf_counter() - t0}
        log("oracle reference %s: %.1f s" % (name, ref_info[name]["seconds"]))
    out["references"] = ref_info
    return out, ref_x


COPY_MIB = 1024


def copy_calibration(mib=COPY_MIB):
    """A plain device copy of known size (the runtime's copy kernel), whose
    counter readings scale FETCH_SIZE / WRITE_SIZE into HBM bytes.  A write of
    another buffer of the same size first evicts the source from the 256 MB
    last-level cache, so the copy really reads HBM."""
    import torch
    a = torch.ones(mib << 18, dtype=torch.float32, device="cuda")
    evict = torch.zeros(mib << 18, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    del evict
    return mib << 20


def summarize_counters(fetch_csv, write_csv, knobs, copy_bytes=COPY_MIB << 20,
                       out_path=TRAFFIC_FILE):
    """Average FETCH_SIZE / WRITE_SIZE (KiB per dispatch) of the working round
    launches from two rocprofv3 --pmc runs taken at the given knobs (the
    --tune string of those runs), scaled by the same counters on the
    calibration copy; adds or replaces the entry for these knobs in out_path
    (profiles/round_kernel_traffic.json)."""
    import csv

    def per_kernel(path, counter):
        rows, copy = [], []
        with open(path) as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                name, v = row.get("Kernel_Name", ""), float(row["Counter_Value"])
                if "k_round" in name:
                    rows.append((int(row.get("Dispatch_Id", 0) or 0), v))
                elif "copyBuffer" in name:
                    copy.append(v)
        return [v for _, v in sorted(rows)], copy

    fa, fc = per_kernel(fetch_csv, "FETCH_SIZE")
    wa, wc = per_kernel(write_csv, "WRITE_SIZE")
    # Launches issued after a solve stopped load their inputs, see the stop and
    # return: they write nothing.  Both runs launch the same sequence, so the
    # write run tells the working launches of both.
    if len(fa) == len(wa):
        keep = [w > 64.0 for w in wa]
        f = [v for v, k in zip(fa, keep) if k]
        w = [v for v, k in zip(wa, keep) if k]
    else:
        f, w = [v for v in fa if v > 64.0], [v for v in wa if v > 64.0]
    fkib, wkib = sum(f) / len(f), sum(w) / len(w)
    # the calibration copy reads and writes copy_bytes: its largest dispatch
    cf = max(fc) * 1024.0 / copy_bytes if fc else 1.0
    cw = max(wc) * 1024.0 / copy_bytes if wc else 1.0
    entry = {"knobs": knobs, "fetch_kib_per_dispatch": fkib / cf,
             "write_kib_per_dispatch": wkib / cw,
             "raw": {"fetch_kib": fkib, "write_kib": wkib, "copy_fetch_factor": cf,
                     "copy_write_factor": cw, "dispatches": [len(f), len(w)]}}
    # one entry per knob setting, all taken on the current kernel sources
    entries = [e for e in load_traffic(out_path).get("entries", []) if e["knobs"] != knobs]
    out = {"kernel_hash": kernel_hash(),
           "entries": sorted(entries + [entry], key=lambda e: [str(k) for k in e["knobs"]])}
    with open(out_path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(entry))
    return entry


def summarize_trace(path):
    """Working-launch durations per kernel from a rocprofv3 kernel trace: the
    launches issued after a solve has stopped return at once (a few us) and
    are listed apart."""
    import csv
    per = {}
    with open(path) as fh:
        for row in csv.DictReader(fh):
            name = row["Kernel_Name"]
            dur = (int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) / 1000.0
            per.setdefault(name, []).append(dur)
    for name, ds in sorted(per.items(), key=lambda kv: -sum(kv[1])):
        work = [d for d in ds if d > 10.0] if ("k_round" in name or "k_pull" in name) else ds
        idle = len(ds) - len(work)
        print("%-70s calls %5d  working %5d  avg_working_us %9.2f  min %8.2f  max %9.2f  "
              "returned-at-once %d" % (name[:70], len(ds), len(work),
                                       sum(work) / max(1, len(work)), min(work or [0]),
                                       max(work or [0]), idle))


def time_steps(fn, steps, warmup):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    outs = [fn() for _ in range(steps)]
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / steps, outs


def bench_ppr_batch(di, G, g, args):
    import numpy as np
    import workloads as wl
    ptr, seeds = wl.ppr_seed_sets(g.n, 256, 100, seed=4)
    tune, fixed = None, None
    if args.batch_tune:  # fixed knobs (profiling runs)
        sc, c, wl_, th = args.batch_tune.split(":")
        fixed = di.make_tune(sc, float(c), int(wl_), threads=int(th))
        tune = di.tune_dict(fixed)
    elif not args.no_autotune:  # tuned on a separate sample of 32 seed sets
        sp, ss = wl.ppr_seed_sets(g.n, 32, 100, seed=40)
        best, _ = di.autotune(G, "batch", d=args.d, tol=1e-6, precision="fp32", seed_ptr=sp,
                              seeds=ss)
        tune = di.tune_dict(best)
    try:
        run = lambda: di.solve_batch(G, ptr, seeds, d=args.d, tol=1e-6, precision="fp32",
                                     tune=fixed)
        t, outs = time_steps(run, 1, 1)
    except di.DiError as e:
        return {"status": "unavailable", "reason": str(e)}
    stats = outs[-1][1]
    # one-at-a-time reference on a sample of 16 vectors at the same tolerance
    t1 = time.perf_counter()
    for b in range(16):
        v = wl.seed_vector(g.n, seeds[ptr[b]:ptr[b + 1]])
        di.solve(G, v=v, d=args.d, tol=1e-6, precision="fp32")
    import torch
    torch.cuda.synchronize()
    solo = (time.perf_counter() - t1) / 16
    # the single solve's byte model summed over the vectors, over the whole batch time
    abytes = float(sum(algorithmic_bytes(g.n, s, "fp32") for s in stats))
    return {"vectors": 256, "tol": 1e-6, "tune": tune, "seconds": t, "vectors_per_s": 256 / t,
            "solo_seconds_per_vector": solo, "speedup_vs_solo": solo * 256 / t,
            "edges_diffused": int(sum(s["edges_diffused"] for s in stats)),
            "rounds_max": int(max(s["rounds"] for s in stats)),
            "rounds_mean": float(np.mean([s["rounds"] for s in stats])),
            "algorithmic_bytes": abytes, "achieved_gbs": abytes / t / 1e9,
            "frac_of_hbm_peak": abytes / t / 1e9 / HBM_PEAK_GBS}


def bench_update(di, G, g, args, tune=None):
    """Graph update (Section 3.2): 1% of the nodes get new out-link lists;
    the converged state of the old graph plus the injected fluid d(P'-P)H is
    resumed on the new graph, against a fresh solve of the new graph.  Every
    solve here uses the knobs tuned on the original graph (tune)."""
    import numpy as np
    import torch
    import workloads as wl
    g1 = wl.modify_graph(g, 0.01, seed=77)
    G1 = di.Graph(g1)
    dt = torch.float32 if args.precision == "fp32" else torch.float64
    reps, t_upd, t_fresh, st_u, st_f = 3, [], [], None, None
    for _ in range(reps):
        F = torch.full((g.n,), (1 - args.d) / g.n, dtype=dt, device="cuda")
        H = torch.zeros(g.n, dtype=torch.float64, device="cuda")
        di.solve(G, d=args.d, tol=args.tol, precision=args.precision, state=(F, H), tune=tune)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        di.inject_update(G, G1, F, H, d=args.d)
        _, st_u = di.solve(G1, d=args.d, tol=args.tol, precision=args.precision, state=(F, H),
                           tune=tune)
        torch.cuda.synchronize()
        t_upd.append(time.perf_counter() - t0)
        t0 = time.perf_counter()
        _, st_f = di.solve(G1, d=args.d, tol=args.tol, precision=args.precision, tune=tune)
        torch.cuda.synchronize()
        t_fresh.append(time.perf_counter() - t0)
    # On-line use: a stream of small changes (0.1% of the nodes each), every
    # one injected into the state left by the previous one and resumed.
    steps, frac = 10, 0.001
    gs, Gs, t_setup = [g], [G], []
    for k in range(steps):
        gs.append(wl.modify_graph(gs[-1], frac, seed=100 + k))
        Gs.append(di.Graph(gs[-1]))
        # one-off per graph, like its residency: the window tables of its first solve
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        di.solve(Gs[-1], d=args.d, tol=args.tol, precision=args.precision, tune=tune,
                 max_rounds=1, allow_notconv=True)
        torch.cuda.synchronize()
        t_setup.append(time.perf_counter() - t0)
    F = torch.full((g.n,), (1 - args.d) / g.n, dtype=dt, device="cuda")
    H = torch.zeros(g.n, dtype=torch.float64, device="cuda")
    di.solve(G, d=args.d, tol=args.tol, precision=args.precision, state=(F, H), tune=tune)
    t_step, t_inj, l_step, r_step = [], [], [], []
    for k in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        di.inject_update(Gs[k], Gs[k + 1], F, H, d=args.d)
        torch.cuda.synchronize()  # to time the injection apart (the call itself does not wait)
        t_inj.append(time.perf_counter() - t0)
        x_u, st_k = di.solve(Gs[k + 1], d=args.d, tol=args.tol, precision=args.precision,
                             state=(F, H), tune=tune)
        torch.cuda.synchronize()
        t_step.append(time.perf_counter() - t0)
        l_step.append(st_k["edges_diffused"])
        r_step.append(st_k["rounds"])
    t0 = time.perf_counter()
    x_f, st_ff = di.solve(Gs[-1], d=args.d, tol=args.tol, precision=args.precision,
                         tune=tune)
    torch.cuda.synchronize()
    t_ff = time.perf_counter() - t0
    l1 = float(torch.sum(torch.abs(x_u - x_f)).item())
    return {"changed_nodes": int(0.01 * g.n), "links_new_graph": g1.m,
            "update_ms": 1e3 * min(t_upd), "fresh_ms": 1e3 * min(t_fresh),
            "speedup": min(t_fresh) / min(t_upd),
            "update_rounds": st_u["rounds"], "update_links": st_u["edges_diffused"],
            "fresh_rounds": st_f["rounds"], "fresh_links": st_f["edges_diffused"],
            "update_residual_l1": st_u["residual_l1"],
            "stream": {"steps": steps, "changed_fraction_per_step": frac,
                       "mean_update_ms": 1e3 * float(np.mean(t_step)),
                       "mean_inject_ms": 1e3 * float(np.mean(t_inj)),
                       "mean_graph_setup_ms": 1e3 * float(np.mean(t_setup)),
                       "max_update_ms": 1e3 * max(t_step),
                       "mean_update_links": float(np.mean(l_step)),
                       "mean_update_rounds": float(np.mean(r_step)),
                       "fresh_rounds_last_graph": st_ff["rounds"],
                       "fresh_ms_last_graph": 1e3 * t_ff,
                       "fresh_links_last_graph": st_ff["edges_diffused"],
                       "l1_update_path_vs_fresh": l1,
                       "bounds_sum": st_k["err_bound_l1"] + st_ff["err_bound_l1"]}}


def bench_paper_replay(di, args):
    """The paper's six simulation scenarios (Section 4.1): links diffused by the
    D-iteration (its elementary steps) and by the power iteration (L per
    product), device times, fp64, same stop rule."""
    import workloads as wl
    rows = {}
    for name in wl.PAPER_SCENARIOS:
        g = wl.paper_scenario(name)
        G = di.Graph(g)
        di.solve(G, d=args.d, tol=args.tol, precision="fp64")
        _, st = di.solve(G, d=args.d, tol=args.tol, precision="fp64")
        # the same knobs, every round in one launch (graphs of at most 128 windows)
        pt = di.make_tune("mean", 1.0, persist=True)
        di.solve(G, d=args.d, tol=args.tol, precision="fp64", tune=pt)
        _, stp = di.solve(G, d=args.d, tol=args.tol, precision="fp64", tune=pt)
        di.power_solve(G, d=args.d, tol=args.tol, precision="fp64")
        _, sp = di.power_solve(G, d=args.d, tol=args.tol, precision="fp64")
        rows[name] = {"n": g.n, "links": g.m, "dangling": g.n_dangling,
                      "diter_links": st["edges_diffused"], "diter_rounds": st["rounds"],
                      "diter_ms": 1e3 * st["seconds"],
                      "diter_one_launch_ms": 1e3 * stp["seconds"],
                      "diter_one_launch_rounds": stp["rounds"],
                      "power_links": sp["rounds"] * g.m, "power_products": sp["rounds"],
                      "power_ms": 1e3 * sp["seconds"],
                      "link_ratio": sp["rounds"] * g.m / max(1, st["edges_diffused"])}
    return rows


def _time_solves(fn, reps):
    """Median wall time of reps calls of fn (each synchronised), and the last
    call's result."""
    import numpy as np
    import torch
    ts, r = [], None
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts)), r


def parse_c1_tune(text):
    """SCHED:C:WLOG[:persist] -> (schedule, c, window_log2, persist)."""
    f = text.split(":")
    if len(f) not in (3, 4) or (len(f) == 4 and f[3] != "persist") or \
            f[0] not in ("mean", "op", "op2"):
        raise SystemExit("--c1-tune takes SCHED:C:WLOG or SCHED:C:WLOG:persist")
    return f[0], float(f[1]), int(f[2]), len(f) == 4


def bench_c1(di, args):
    """The small graph: N = 10^4, mean degree 8, 10% dangling, fp64 fluid,
    ||F||_1 < 1e-10, against the fp64 power iteration to the same stop.
    Returns (summary, {result name: host x})."""
    import workloads as wl
    g = wl.recipe("pagerank-10k")
    G = di.Graph(g)
    tol = 1e-10
    tune = None
    if args.c1_tune:  # fixed knobs (profiling runs)
        sched, c, wlog, persist = parse_c1_tune(args.c1_tune)
        tune = di.make_tune(sched, c, wlog, persist=persist)
    elif not args.no_autotune:
        tune, _ = di.autotune(G, "solve", d=0.85, tol=tol, precision="fp64")
    for _ in range(3):  # warm-up
        di.solve(G, d=0.85, tol=tol, precision="fp64", tune=tune)
        di.power_solve(G, d=0.85, tol=tol, precision="fp64")
    t, (x, st) = _time_solves(lambda: di.solve(G, d=0.85, tol=tol, precision="fp64", tune=tune), 20)
    tp, (xp, sp) = _time_solves(lambda: di.power_solve(G, d=0.85, tol=tol, precision="fp64"), 20)
    out = {"workload": "pagerank-10k", "n": g.n, "links": g.m, "dangling": g.n_dangling,
           "d": 0.85, "tol": tol, "precision": "fp64",
           "tune": di.tune_dict(tune) if tune is not None else None,
           "diter": {"ms_per_solve": 1e3 * t, "device_ms": 1e3 * st["seconds"],
                     "rounds": st["rounds"], "edges_diffused": st["edges_diffused"],
                     "edges_diffused_per_s": st["edges_diffused"] / t,
                     "residual_l1": st["residual_l1"], "err_bound_l1": st["err_bound_l1"]},
           "power": {"ms_per_solve": 1e3 * tp, "device_ms": 1e3 * sp["seconds"],
                     "products": sp["rounds"], "link_visits": sp["rounds"] * g.m,
                     "residual_l1": sp["residual_l1"], "err_bound_l1": sp["err_bound_l1"]},
           "speedup_of_diter": tp / t}
    return out, {"c1_diter": x.cpu().numpy(), "c1_power": xp.cpu().numpy()}, g


def bench_c3(di, args):
    """The web-shaped graph: N = 2e7, ~3e8 links, host blocks of 1000 ids with
    80% of the links inside, 15% dangling; fp32 fluid, ||F||_1 < 1e-8, for
    d = 0.85 and 0.90, against the power iteration (both variants) to the same
    stop.  Returns (summary, {result name: host x}, graph)."""
    import workloads as wl
    log("generating web-20m")
    t0 = time.perf_counter()
    g = wl.recipe("web-20m")
    gen_s = time.perf_counter() - t0
    t0 = time.perf_counter()
    G = di.Graph(g)
    import torch
    torch.cuda.synchronize()
    res_s = time.perf_counter() - t0
    log("web-20m n=%d links=%d (generated in %.1f s, resident in %.1f s)" % (g.n, g.m, gen_s, res_s))
    tol, out, xs = 1e-8, {}, {}
    for d in (0.85, 0.90):
        tune = None
        if not args.no_autotune:
            tune, _ = di.autotune(G, "solve", d=d, tol=tol, precision="fp32")
        di.solve(G, d=d, tol=tol, precision="fp32", tune=tune)
        t, (x, st) = _time_solves(lambda: di.solve(G, d=d, tol=tol, precision="fp32", tune=tune), 3)
        _, (_, stt) = _time_solves(lambda: di.solve(G, d=d, tol=tol, precision="fp32", tune=tune,
                                                    timing=True), 1)
        comp = {}
        for prec in ("fp32", "fp64"):
            di.power_solve(G, d=d, tol=tol, precision=prec)
            tp, (xp, sp) = _time_solves(lambda: di.power_solve(G, d=d, tol=tol, precision=prec), 2)
            _, spt = di.power_solve(G, d=d, tol=tol, precision=prec, timing=True)
            comp[prec] = {"ms_per_solve": 1e3 * tp, "products": sp["rounds"],
                          "kernel_us_per_product": 1e6 * spt["kernel_seconds"] /
                          max(1, spt["kernel_launches"]),
                          "residual_l1": sp["residual_l1"]}
            xs["c3_d%.2f_power_%s" % (d, prec)] = xp.cpu().numpy()
            del xp
        best = min(comp, key=lambda k: comp[k]["ms_per_solve"])
        key = "d=%.2f" % d
        out[key] = {"tune": di.tune_dict(tune) if tune is not None else None,
                    "diter": {"ms_per_solve": 1e3 * t, "rounds": st["rounds"],
                              "edges_diffused": st["edges_diffused"],
                              "edges_diffused_per_s": st["edges_diffused"] / t,
                              "round_kernel_us": 1e6 * stt["kernel_seconds"] /
                              max(1, stt["kernel_launches"]),
                              "residual_l1": st["residual_l1"],
                              "err_bound_l1": st["err_bound_l1"]},
                    "power": comp, "best_power_variant": best,
                    "speedup_of_diter": comp[best]["ms_per_solve"] / (1e3 * t)}
        xs["c3_d%.2f_diter" % d] = x.cpu().numpy()
        del x
    del G
    return ({"workload": "web-20m", "n": g.n, "links": g.m, "dangling": g.n_dangling,
             "tol": tol, "precision": "fp32 fluid, fp64 history", "generate_s": gen_s,
             "residency_s": res_s, "by_d": out}, xs, g)


SERVE_GRAPHS = ("serve-100k", "serve-500k", "serve-1m", "serve-5m")
SERVE_TOLS = (1e-4, 1e-6, 1e-8)


def _run_stream(di, srv, gids, graphs, t, gi, sizes, tol, sub, d, label):
    """Submit requests at their arrival times (open loop); returns the results
    in submission order and the wall time of the submission phase."""
    import numpy as np
    import workloads as wl
    seeds = [wl.request_seeds(graphs[g].n, int(s), int(u)) for g, s, u in zip(gi, sizes, sub)]
    rids = []
    t0 = time.perf_counter()
    next_log = 10.0
    for k in range(len(t)):
        while True:
            now = time.perf_counter() - t0
            if now >= t[k]:
                break
            if t[k] - now > 2e-4:
                time.sleep(min(t[k] - now - 1e-4, 0.01))
        rids.append(srv.submit(gids[gi[k]], seeds[k], d=d, tol=float(tol[k])))
        if now > next_log:
            log("%s: %.0f s, %d submitted, %s" % (label, now, k + 1, srv.stats()["active"]))
            next_log += 10.0
    sub_s = time.perf_counter() - t0
    res = []
    for k, rid in enumerate(rids):
        r = srv.wait(rid, 120.0)
        if r is None:
            raise RuntimeError("request %d did not finish within 120 s" % k)
        res.append(r)
    return res, sub_s


def run_section_child(name, args, forward):
    """Runs one section of this script in a child process (same interpreter,
    same flags as given in `forward`) and returns its result; a crash or a
    time-out there loses that section only, reported as an error."""
    import subprocess
    cmd = [sys.executable, os.path.abspath(__file__), "--section", name] + forward
    log("section %s in a child process" % name)
    try:
        p = subprocess.run(cmd, stdout=subprocess.PIPE, text=True, timeout=1200)
    except subprocess.TimeoutExpired:
        return {"error": "section %s timed out" % name}
    lines = [ln for ln in p.stdout.splitlines() if ln.startswith("{")]
    if p.returncode != 0 or not lines:
        return {"error": "section %s exited with status %d" % (name, p.returncode)}
    return json.loads(lines[-1])["result"]


def serve_forward(args):
    """The command-line flags of the serving section."""
    f = ["--d", repr(args.d), "--serve-rate", repr(args.serve_rate),
         "--serve-seconds", repr(args.serve_seconds),
         "--serve-sustained-seconds", repr(args.serve_sustained_seconds),
         "--serve-warmup", repr(args.serve_warmup), "--serve-burst", str(args.serve_burst),
         "--serve-solo", str(args.serve_solo), "--serve-hbm-gib", str(args.serve_hbm_gib)]
    return f + (["--no-autotune"] if args.no_autotune else [])


def bench_serve(di, args):
    """Continuous-batching server on the four resident serving graphs: an
    open-loop Poisson stream (latency percentiles, achieved rate), a burst of
    requests submitted at once (capacity), and the same requests one at a time
    (a server with one slot) as the baseline the batching has to beat."""
    import numpy as np
    import workloads as wl
    graphs = [wl.recipe(r) for r in SERVE_GRAPHS]
    G = [di.Graph(g) for g in graphs]
    tunes = {}
    if not args.no_autotune:  # per graph, on 16 seed sets drawn like the stream's
        for name, g, x in zip(SERVE_GRAPHS, graphs, G):
            rng = np.random.default_rng(7)
            sz = np.clip(np.floor(np.exp(rng.uniform(0, np.log(1001), 16))), 1, 1000).astype(int)
            sets = [wl.request_seeds(g.n, int(k), int(rng.integers(1 << 62))) for k in sz]
            ptr = np.concatenate([[0], np.cumsum([len(q) for q in sets])]).astype(np.int64)
            best, _ = di.autotune(x, "batch", d=args.d, tol=1e-6, precision="fp32", seed_ptr=ptr,
                                  seeds=np.concatenate(sets))
            tunes[name] = di.tune_dict(best)
            log("serve autotune %s: %s" % (name, tunes[name]))
    srv = di.Server(hbm_budget_bytes=args.serve_hbm_gib << 30, max_slots=256, topk=100)
    gids = [srv.add_graph(x) for x in G]
    caps = srv.stats()["hbm_in_use"]
    dur = args.serve_warmup + args.serve_seconds
    t, gi, sizes, tol, sub = wl.poisson_stream(args.serve_rate, dur, len(graphs), 1000,
                                               SERVE_TOLS, seed=5)
    log("serve: %d requests over %.1f s at %.0f/s" % (len(t), dur, args.serve_rate))
    res, sub_s = _run_stream(di, srv, gids, graphs, t, gi, sizes, tol, sub, args.d, "serve")
    meas = [r for r, tk in zip(res, t) if tk >= args.serve_warmup]
    ok = sum(r["status"] == 0 for r in res)
    lat = np.array([r["t_done"] - r["t_submit"] for r in meas])
    t_first = min(r["t_submit"] for r in meas)
    t_last = max(r["t_done"] for r in meas)
    achieved = len(meas) / (t_last - t_first)
    per_graph = {}
    for g in range(len(graphs)):
        lg = np.array([r["t_done"] - r["t_submit"] for r, tk, q in zip(res, t, gi)
                       if tk >= args.serve_warmup and q == g])
        if len(lg):
            rg = [r for r, q in zip(res, gi) if q == g]
            per_graph[SERVE_GRAPHS[g]] = {"requests": int(len(lg)),
                                          "p50_ms": 1e3 * float(np.percentile(lg, 50)),
                                          "p99_ms": 1e3 * float(np.percentile(lg, 99)),
                                          "mean_rounds": float(np.mean([r["rounds"] for r in rg])),
                                          "mean_links": float(np.mean([r["edges_diffused"]
                                                                       for r in rg]))}
    srv.close()

    # capacity: a burst of requests with the stream's mix, all submitted at once
    nb_ = args.serve_burst
    tb, gib, szb, tolb, subb = wl.poisson_stream(1e9, 1.0, len(graphs), 1000, SERVE_TOLS, seed=6)
    tb, gib, szb, tolb, subb = (x[:nb_] for x in (tb, gib, szb, tolb, subb))
    srv = di.Server(hbm_budget_bytes=args.serve_hbm_gib << 30, max_slots=256, topk=100)
    gids = [srv.add_graph(x) for x in G]
    t0 = time.perf_counter()
    rb, _ = _run_stream(di, srv, gids, graphs, np.zeros(nb_), gib, szb, tolb, subb, args.d, "burst")
    burst_s = time.perf_counter() - t0
    srv.close()

    # one at a time: the first requests of the burst through a one-slot server
    ns = args.serve_solo
    srv = di.Server(hbm_budget_bytes=args.serve_hbm_gib << 30, max_slots=1, topk=100)
    gids = [srv.add_graph(x) for x in G]
    t0 = time.perf_counter()
    rs, _ = _run_stream(di, srv, gids, graphs, np.zeros(ns), gib[:ns], szb[:ns], tolb[:ns],
                        subb[:ns], args.d, "solo")
    solo_s = time.perf_counter() - t0
    srv.close()
    # the same request alone and in the burst: top-k values within both bounds
    worst = 0.0
    for a, b in zip(rs, rb[:ns]):
        va = dict(zip(a["top_ids"].tolist(), a["top_x"].tolist()))
        vb = dict(zip(b["top_ids"].tolist(), b["top_x"].tolist()))
        bound = a["err_bound_l1"] + b["err_bound_l1"]
        for i in set(va) & set(vb):
            worst = max(worst, abs(va[i] - vb[i]) - bound)
    capacity = nb_ / burst_s
    solo_qps = ns / solo_s

    # the same kind of stream at 70% of the measured capacity: the latencies
    # the server gives while it keeps up
    sustained = None
    if achieved < 0.95 * args.serve_rate:
        rate = 0.7 * capacity
        srv = di.Server(hbm_budget_bytes=args.serve_hbm_gib << 30, max_slots=256, topk=100)
        gids = [srv.add_graph(x) for x in G]
        dur2 = args.serve_warmup + args.serve_sustained_seconds
        ts, gs, ss, tl, us = wl.poisson_stream(rate, dur2, len(graphs), 1000, SERVE_TOLS, seed=8)
        log("serve at %.0f/s: %d requests" % (rate, len(ts)))
        r2, _ = _run_stream(di, srv, gids, graphs, ts, gs, ss, tl, us, args.d, "serve70")
        srv.close()
        m2 = [r for r, tk in zip(r2, ts) if tk >= args.serve_warmup]
        l2 = np.array([r["t_done"] - r["t_submit"] for r in m2])
        ach2 = len(m2) / (max(r["t_done"] for r in m2) - min(r["t_submit"] for r in m2))
        sustained = {"rate_per_s": rate, "measured_s": args.serve_sustained_seconds,
                     "requests": len(r2), "measured_requests": len(m2),
                     "achieved_qps": ach2, "p50_ms": 1e3 * float(np.percentile(l2, 50)),
                     "p99_ms": 1e3 * float(np.percentile(l2, 99)),
                     "ok": sum(r["status"] == 0 for r in r2)}
    return {
        "graphs": {n: {"n": g.n, "links": g.m} for n, g in zip(SERVE_GRAPHS, graphs)},
        "hbm_budget_gib": args.serve_hbm_gib, "slot_bytes_total": caps, "tune": tunes,
        "stream": {"rate_per_s": args.serve_rate, "warmup_s": args.serve_warmup,
                   "measured_s": args.serve_seconds, "requests": len(res),
                   "measured_requests": len(meas), "ok": ok,
                   "submit_wall_s": sub_s, "achieved_qps": achieved,
                   "sustained": bool(achieved >= 0.95 * args.serve_rate),
                   "p50_ms": 1e3 * float(np.percentile(lat, 50)),
                   "p99_ms": 1e3 * float(np.percentile(lat, 99)),
                   "per_graph": per_graph},
        "burst": {"requests": nb_, "seconds": burst_s, "capacity_qps": capacity,
                  "ok": sum(r["status"] == 0 for r in rb)},
        "one_at_a_time": {"requests": ns, "seconds": solo_s, "qps": solo_qps},
        "speedup_vs_one_at_a_time": capacity / solo_qps,
        "saturation_qps": None if achieved >= 0.95 * args.serve_rate else capacity,
        "stream_at_70pct_capacity": sustained,
        "alone_vs_mix_max_excess": worst,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="powerlaw-1m")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp64"])
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--d", type=float, default=0.85)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ppr", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-update", action="store_true")
    ap.add_argument("--no-replay", action="store_true")
    ap.add_argument("--no-c1", action="store_true", help="skip the 10^4-node fp64 solve")
    ap.add_argument("--no-c3", action="store_true", help="skip the 2e7-node web-shaped graph")
    ap.add_argument("--no-autotune", action="store_true",
                    help="library default knobs instead of di_autotune's choice")
    ap.add_argument("--section", choices=["ppr", "serve", "update", "replay", "c1", "c3"],
                    help="run only this part and print its JSON (profiling runs)")
    ap.add_argument("--tune", metavar="SCHED:C:WLOG:THREADS",
                    help="fixed knobs for the single solve instead of autotuning (profiling runs)")
    ap.add_argument("--c1-tune", metavar="SCHED:C:WLOG[:persist]",
                    help="fixed knobs for the 10^4-node solve instead of autotuning (profiling runs)")
    ap.add_argument("--batch-tune", metavar="SCHED:C:WLOG:THREADS",
                    help="fixed knobs for the batch instead of autotuning (profiling runs)")
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-seconds", type=float, default=5.0,
                    help="measured seconds of the stream at the configured rate (which "
                         "saturates the server: its backlog grows)")
    ap.add_argument("--serve-sustained-seconds", type=float, default=60.0,
                    help="measured seconds of the stream at 70%% of the measured capacity")
    ap.add_argument("--serve-warmup", type=float, default=1.0)
    ap.add_argument("--serve-burst", type=int, default=2000)
    ap.add_argument("--serve-solo", type=int, default=100)
    ap.add_argument("--serve-hbm-gib", type=int, default=32)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a 1 GiB device copy (counter calibration)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write profiles/round_kernel_traffic.json from two --pmc runs")
    ap.add_argument("--summarize-trace", metavar="KERNEL_TRACE_CSV",
                    help="print per-kernel durations of the working launches from a trace")
    args = ap.parse_args()
    if args.summarize_counters:
        if not args.tune:
            sys.exit("--summarize-counters needs the --tune knobs the counter runs used")
        sc, c, wl_, th = args.tune.split(":")
        summarize_counters(*args.summarize_counters,
                           knobs=launch_knobs({"schedule": sc, "c": float(c),
                                               "window_log2": int(wl_), "threads": int(th)}))
        return
    if args.summarize_trace:
        summarize_trace(args.summarize_trace)
        return
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(--gpus %d, WORLD_SIZE %d)" % (args.gpus, world), file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads as wl
    from paper_1202_6158_amd import di
    torch.cuda.set_device(0)

    g = G = None
    if args.section in (None, "ppr", "update"):
        log("generating", args.workload)
        g = wl.recipe(args.workload)
        G = di.Graph(g)
        log("graph n=%d links=%d dangling=%d" % (g.n, g.m, g.n_dangling))
    if args.section:
        part = {"ppr": lambda: bench_ppr_batch(di, G, g, args),
                "serve": lambda: bench_serve(di, args),
                "update": lambda: bench_update(di, G, g, args, None if args.no_autotune else
                                               di.autotune(G, "solve", d=args.d, tol=args.tol,
                                                           precision=args.precision)[0]),
                "replay": lambda: bench_paper_replay(di, args),
                "c1": lambda: bench_c1(di, args)[0],
                "c3": lambda: bench_c3(di, args)[0]}[args.section]()
        print(json.dumps({"section": args.section, "result": part}), flush=True)
        return

    # ---- autotuner: the knobs every later solve on this graph uses
    tune_info = None
    fixed = None
    solve_tune = None  # the knobs the solves below use (also the update section's)
    if args.tune:
        sc, c, wl_, th = args.tune.split(":")
        fixed = di.make_tune(sc, float(c), int(wl_), threads=int(th))
        tune_info = {"best": di.tune_dict(fixed), "fixed": True}
    elif not args.no_autotune:
        t0 = time.perf_counter()
        best, trials = di.autotune(G, "solve", d=args.d, tol=args.tol, precision=args.precision)
        solve_tune = best
        ok = [t for t in trials if t["status"] == 0]
        tune_info = {"best": di.tune_dict(best), "candidates": len(trials),
                     "default_ms": 1e3 * trials[0]["seconds"],
                     "best_ms": 1e3 * min(t["seconds"] for t in ok),
                     "tuning_s": time.perf_counter() - t0}
        log("autotune: %s (%.3f ms vs %.3f ms default)" % (tune_info["best"], tune_info["best_ms"],
                                                          tune_info["default_ms"]))

    # ---- D-iteration (the measured step): K un-instrumented solves give the
    # throughput; the same K solves again with per-launch HIP events (the
    # runtime stamps each round kernel's begin/end) give its launch durations.
    solve = lambda timing: di.solve(G, d=args.d, tol=args.tol, precision=args.precision,
                                    timing=timing, tune=fixed)
    sec, outs = time_steps(lambda: solve(False), args.steps, args.warmup)
    x_di = outs[-1][0]
    sec_timed, touts = time_steps(lambda: solve(True), args.steps, 0)
    stats = [s for _, s in touts]
    dev_ms = 1e3 * float(np.mean([s["seconds"] for _, s in outs]))
    ksec = float(np.sum([s["kernel_seconds"] for s in stats]))
    kl = int(np.sum([s["kernel_launches"] for s in stats]))
    abytes = float(np.mean([algorithmic_bytes(g.n, s, args.precision) for s in stats]))
    launches_per_solve = kl / len(stats)
    per_launch_bytes = abytes / launches_per_solve
    per_launch_sec = ksec / kl
    achieved = per_launch_bytes / per_launch_sec / 1e9
    st = outs[-1][1]
    # the same solve with x returned into host memory (a copy over the bus
    # inside every step): the rate a caller with host buffers sees
    hsec, _ = time_steps(lambda: di.solve(G, d=args.d, tol=args.tol, precision=args.precision,
                                          tune=fixed, host=True), max(2, args.steps // 2), 1)
    log("diter: %.3f ms/solve (device %.3f ms), %d rounds, %.3g links, residual %.2e"
        % (sec * 1e3, dev_ms, st["rounds"], st["edges_diffused"], st["residual_l1"]))

    # ---- comparator: GPU power iteration, both precision variants
    comp = {}
    for prec in ("fp64", "fp32"):
        # timed like the D-iteration: plain launches (the per-launch events of
        # an instrumented solve add time between launches)
        pstep = lambda: di.power_solve(G, d=args.d, tol=args.tol, precision=prec)
        psec, pouts = time_steps(pstep, max(2, args.steps // 2), 1)
        _, ps = di.power_solve(G, d=args.d, tol=args.tol, precision=prec, timing=True)
        comp[prec] = {"ms_per_solve": psec * 1e3, "products": ps["rounds"],
                      "kernel_us_per_product": 1e6 * ps["kernel_seconds"] / max(1, ps["kernel_launches"]),
                      "residual_l1": pouts[-1][1]["residual_l1"], "x": pouts[-1][0]}
    best = min(comp, key=lambda k: comp[k]["ms_per_solve"])
    l1_di_vs_power = float(torch.sum(torch.abs(x_di - comp["fp64"]["x"])).item())
    x_pow64 = comp["fp64"]["x"].cpu().numpy()
    for k in comp:
        comp[k].pop("x")
    log("power: fp64 %.3f ms, fp32 %.3f ms" % (comp["fp64"]["ms_per_solve"], comp["fp32"]["ms_per_solve"]))

    out = {
        "metric": METRIC,
        "value": 1.0 / sec,
        "unit": "solves/s (PageRank to L1 residual %g)" % args.tol,
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32" if args.precision == "fp32" else "f64",
        "dtype_detail": ("fp32 fluid and pushes; fp64 window accumulation, history, residual "
                         "and normalisation") if args.precision == "fp32" else "fp64 throughout",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": g.n, "links": g.m, "dangling": g.n_dangling,
                   "d": args.d, "tol": args.tol, "V": "uniform",
                   "recipe": wl.RECIPES.get(args.workload)},
        "tune": tune_info,
        "time_to_residual_ms": sec * 1e3,
        "device_ms_per_solve": dev_ms,
        "ms_per_solve_with_launch_events": sec_timed * 1e3,
        "host_buffers": {"ms_per_solve": hsec * 1e3, "solves_per_s": 1.0 / hsec,
                         "note": "x (fp64, n entries) copied into host memory inside every "
                                 "step; not the headline value"},
        "rounds": st["rounds"], "nodes_diffused": st["nodes_diffused"],
        "edges_diffused": st["edges_diffused"],
        "edges_diffused_per_s": st["edges_diffused"] / sec,
        "residual_l1": st["residual_l1"], "err_bound_l1": st["err_bound_l1"],
        "mass_drift": st["mass_drift"],
        "comparator": {"kind": "GPU power iteration (pull over in-links), same stop rule",
                       "best_variant": best, "variants": comp,
                       "speedup_of_diter": comp[best]["ms_per_solve"] / (sec * 1e3),
                       "l1_diter_vs_power_fp64": l1_di_vs_power},
        "roofline": {"kernel": "k_round (one D-iteration round)", "bound": "hbm",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic(tune_info["best"] if tune_info else None),
                     "algorithmic_bytes_per_launch": per_launch_bytes,
                     "avg_launch_us": per_launch_sec * 1e6,
                     "launches_per_solve": launches_per_solve,
                     "timing": "hipExtLaunchKernel begin/end events on the solve's stream, "
                               "%d launches over %d solves" % (kl, len(stats))},
    }
    # results whose L1 error against the oracle is reported (host copies)
    results = {"c2_diter": x_di.cpu().numpy(), "c2_power_fp64": x_pow64}
    refs = [("c2", g, args.d, 1e-13, None)]
    if not args.no_c1:
        out["c1"], xs1, g1 = bench_c1(di, args)
        results.update(xs1)
        refs.append(("c1", g1, 0.85, 0.0, None))
        log("c1: diter %.3f ms, power %.3f ms" % (out["c1"]["diter"]["ms_per_solve"],
                                                  out["c1"]["power"]["ms_per_solve"]))
    if not args.no_ppr:
        out["ppr_batch"] = bench_ppr_batch(di, G, g, args)
    if not args.no_update:
        out["update"] = bench_update(di, G, g, args, fixed if fixed is not None else solve_tune)
    if not args.no_replay:
        out["paper_replay"] = bench_paper_replay(di, args)
    if not args.no_serve:
        # in a process of its own: four engine threads and their streams, the
        # longest section; a failure there must not cost the other results
        out["serve"] = run_section_child("serve", args, serve_forward(args))
    if not args.no_c3:
        del G
        torch.cuda.empty_cache()
        out["c3"], xs3, g3 = bench_c3(di, args)
        results.update(xs3)
        for d3 in (0.85, 0.90):
            refs.append(("c3_d%.2f" % d3, g3, d3, 1e-10, None))
        for k, v in out["c3"]["by_d"].items():
            log("c3 %s: diter %.1f ms, power %.1f ms" % (k, v["diter"]["ms_per_solve"],
                                                        v["power"][v["best_power_variant"]]
                                                        ["ms_per_solve"]))
    if args.copy_calibration:
        out["copy_calibration_bytes"] = copy_calibration()
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        out["cpu_baseline"], ref_x = cpu_baseline(g, args.d, args.tol, args.cpu_seconds, refs)
        # L1 error of every reported result against the oracle's fp64 limit
        l1 = {}
        for name, x in results.items():
            ref = next(ref_x[r] for r in sorted(ref_x, key=len, reverse=True)
                       if name.startswith(r + "_"))
            l1[name] = float(np.abs(x - ref).sum())
        out["l1_vs_oracle"] = l1
        out["comparator"]["l1_power_fp64_vs_oracle"] = l1["c2_power_fp64"]
        out["l1_vs_oracle_headline"] = l1["c2_diter"]
        if "c1" in out:
            out["c1"]["diter"]["l1_vs_oracle"] = l1["c1_diter"]
            out["c1"]["power"]["l1_vs_oracle"] = l1["c1_power"]
        if "c3" in out:
            for d3 in (0.85, 0.90):
                e = out["c3"]["by_d"]["d=%.2f" % d3]
                e["diter"]["l1_vs_oracle"] = l1["c3_d%.2f_diter" % d3]
                for prec in ("fp32", "fp64"):
                    e["power"][prec]["l1_vs_oracle"] = l1["c3_d%.2f_power_%s" % (d3, prec)]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
