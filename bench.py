"""Benchmark: LOWD on the Chung-Lu power-law workload (n = 1M nodes, ~10M
unit-weight edges, degree exponent 2.1, a planted 500-node block of pair
density 0.3), FP64 state, no pruning, solved to a 1e-6 relative density
gap.  Other workloads (--workload): chunglu4m (4M nodes, 64M lognormal
edges, FP32 + compensated loads against FP64), rmat24 (R-MAT scale 24,
pruned by Algorithm 2, then LOWD on the pruned graph) and batch4096 (4096
small graphs in the batched form, converged graphs retired).

One step = one whole solve on the GPU from Algorithm 1's initial state:
reset the fractions and loads, then sweep (the phase schedule is built once
per graph, before timing), checking every few sweeps with the extraction
(sort, prefix densities) and the dual bound D = max load, until
(D - rho) / rho <= 1e-6.  The inputs are resident in HBM before timing.

Printed: one JSON line with edge-updates/s over the timed steps (checks
included), the HBM roofline of the sweep measured with HIP events on the
stream the sweeps run on, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE = os.path.join(ROOT, "profiles", "sweep_chunglu_1M_10M_f64.md")
# the sources that decide the sweep's kernels and memory layout
SWEEP_SOURCES = ["paper_2307_15969_amd/csrc/k_sweep.hip", "paper_2307_15969_amd/csrc/sweep_state.h",
                 "paper_2307_15969_amd/csrc/schedule.cpp", "paper_2307_15969_amd/csrc/lowd_internal.h"]


def profiled_traffic():
    """HBM bytes per sweep from the committed FETCH_SIZE/WRITE_SIZE summary,
    or None when the sweep sources changed since the counters were taken
    (the summary records a hash of those sources)."""
    import hashlib
    try:
        text = open(PROFILE).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for p in SWEEP_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    fields = dict(l.split(": ", 1) for l in text.splitlines()
                  if l.startswith(("traffic_bytes_per_sweep: ", "sources_sha256_16: ")))
    if fields.get("sources_sha256_16", "").strip() != h.hexdigest()[:16]:
        return None
    return int(fields["traffic_bytes_per_sweep"])


def sweep_bytes(n: int, m: int, x_bytes: int = 8, w_bytes: int = 0, l_bytes: int = 8) -> int:
    """Algorithmic bytes of one sweep: every edge reads its two endpoint ids
    (8 B), reads and writes its fraction, reads its weight; every node's load
    is read and written once."""
    return m * (8 + 2 * x_bytes + w_bytes) + n * 2 * l_bytes


def cpu_baseline(g, seconds: float = 12.0) -> dict:
    """The FP64 oracle (sequential, one core) on a bounded sample: its own
    schedule, init, then as many full sweeps of the same graph as fit in
    about `seconds`."""
    import oracle
    oracle.build(force=False)
    t0 = time.perf_counter()
    _, _, order, _ = oracle.schedule(g.n, g.src, g.dst, 16)
    t_sched = time.perf_counter() - t0
    x, L = oracle.init(g.n, g.src, g.dst, g.w)
    sweeps = 0
    t0 = time.perf_counter()
    while True:
        oracle.sweep(g.n, g.src, g.dst, g.w, order, 1, x, L)
        sweeps += 1
        el = time.perf_counter() - t0
        if el >= seconds or sweeps >= 200:
            break
    rate = g.m * sweeps / el
    return {"value": rate, "unit": "edge-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{sweeps} full sweeps of the same {g.m}-edge graph in schedule order "
                      f"({el:.1f} s; schedule build {t_sched:.1f} s not included)"}


WORKLOADS = {
    "chunglu1m": "Chung-Lu n=1M, ~10M unit edges, beta 2.1, planted 500-node block p=0.3",
    "chunglu4m": "Chung-Lu n=4M, ~64M lognormal(0,1) edges (float32), beta 2.1, planted block",
    "rmat24": "R-MAT scale 24, edge factor 16, (.57,.19,.19,.05), pruned by Algorithm 2",
    "batch4096": "4096 Chung-Lu graphs (beta 2.3), edges log-uniform in [100, 50000], "
                 "planted blocks of 5-40 nodes",
    "uniform": "diagnostic: 2^28 uniform random pairs on 2^25 nodes (max degree ~45, few wide "
               "phases); sweeps only",
}


def single_solve(sv, stream, tol, check_every, ev_a, ev_b):
    """reset, then sweep/check until the gap tolerance; returns (sweeps,
    seconds spent in sweeps measured with events on the sweep stream, final
    extraction).  The sweeps between checks follow lowd.next_check: at most
    check_every, fewer when the gap's decay predicts the tolerance sooner;
    as in lowd.solve, the first check comes after the first check_every
    sweeps, and a check extracts only when the largest load does not
    certify the best set so far (lowd.certify)."""
    import paper_2307_15969_amd as lowd
    sv.reset(stream)
    sweeps = 0
    sweep_s = 0.0
    ex = None
    gap = float("inf")
    hist = []
    while gap > tol:
        k = lowd.next_check(hist, tol, check_every)
        ev_a.record(stream)
        sv.iterate(k, stream)
        ev_b.record(stream)
        ev_b.synchronize()
        sweep_s += ev_a.elapsed_time(ev_b) / 1e3
        sweeps += k
        ex, gap = lowd.certify(sv, ex, tol, stream)
        hist.append((sweeps, gap))
        if sweeps > 20000:
            raise RuntimeError("no convergence within 20000 sweeps")
    return sweeps, sweep_s, ex


def timed_single(sv, m, args, stream, torch, label):
    ev_a = torch.cuda.Event(enable_timing=True)
    ev_b = torch.cuda.Event(enable_timing=True)
    for i in range(args.warmup):
        s_, _, ex = single_solve(sv, stream, args.tol, args.check_every, ev_a, ev_b)
        print(f"[bench] {label} warmup {i}: {s_} sweeps, gap {ex['gap']:.3e}, "
              f"density {ex['num']}/{ex['den']}", flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot_sweeps, tot_sweep_s, last = 0, 0.0, None
    for i in range(args.steps):
        s_, ss, ex = single_solve(sv, stream, args.tol, args.check_every, ev_a, ev_b)
        tot_sweeps += s_
        tot_sweep_s += ss
        last = (s_, ex)
        print(f"[bench] {label} step {i}: {s_} sweeps, gap {ex['gap']:.3e}", flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    return dict(elapsed=elapsed, sweeps=tot_sweeps, sweep_s=tot_sweep_s, last_sweeps=last[0],
                ex=last[1], value=m * tot_sweeps / elapsed,
                per_sweep_s=tot_sweep_s / max(tot_sweeps, 1))


def density_str(ex, weighted=False):
    """the extracted density: the exact rational for unit weights, else the
    FP64 weight sum over the node count"""
    if weighted:
        return f"{ex['num_w']!r}/{ex['den']}"
    return f"{ex['num']}/{ex['den']}"


def base_line(args, metric_value, ms_per_step, dtype, config):
    return {
        "metric": "LOWD edge-updates/s + % HBM roofline; time to density within 1e-6 of optimum",
        "value": metric_value,
        "unit": "edge-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": config,
    }


def roofline(bytes_per_unit, seconds_per_unit, kernel, traffic=None):
    achieved = bytes_per_unit / seconds_per_unit / 1e9
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic, "kernel": kernel,
            "algorithmic_bytes": bytes_per_unit}


def run_chunglu1m(args, torch, lowd, synth):
    t0 = time.perf_counter()
    g = synth.workload(1, seed=args.seed)
    print(f"[bench] workload {g.name}: n={g.n} m={g.m} generated in "
          f"{time.perf_counter() - t0:.1f}s", flush=True)
    src = torch.from_numpy(g.src).cuda()
    dst = torch.from_numpy(g.dst).cuda()
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    sv = lowd.Solver(g.n, src, dst, None, args.state or "f64", star_max=16)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    info = sv.info()
    print(f"[bench] setup (validation, schedule, CSR, init) {t_setup:.2f}s info {info}", flush=True)
    state = args.state or "f64"
    r = timed_single(sv, g.m, args, stream, torch, state)
    xb, lb = (8, 8) if state == "f64" else (4, 8)
    out = base_line(args, r["value"], r["elapsed"] / args.steps * 1e3, state,
                    {"workload": g.name + " (" + WORKLOADS["chunglu1m"] + "), " + state.upper() +
                     ", no pruning, to 1e-6 gap", "n": g.n, "m": g.m, "star_max": 16,
                     "check_every": args.check_every, "seed": args.seed})
    out.update({
        "time_to_1e-6_ms": r["elapsed"] / args.steps * 1e3,
        "sweeps_to_1e-6": r["last_sweeps"],
        "density": density_str(r["ex"]),
        "sweep_ms": r["per_sweep_s"] * 1e3,
        "sweep_edge_updates_per_s": g.m / r["per_sweep_s"],
        "setup_s": t_setup,
        "schedule": info,
        "roofline": roofline(sweep_bytes(g.n, g.m, xb, 0, lb), r["per_sweep_s"],
                             "one sweep (the HIP graph of phase kernels + single-workgroup tiers)",
                             profiled_traffic() if state == "f64" else None),
    })
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, args.cpu_seconds)
    return out


def run_chunglu4m(args, torch, lowd, synth):
    t0 = time.perf_counter()
    g = synth.workload(2, seed=args.seed)
    print(f"[bench] workload {g.name}: n={g.n} m={g.m} generated in "
          f"{time.perf_counter() - t0:.1f}s", flush=True)
    src = torch.from_numpy(g.src).cuda()
    dst = torch.from_numpy(g.dst).cuda()
    w = torch.from_numpy(g.w).cuda()
    stream = torch.cuda.current_stream()
    res = {}
    for state in ("f32k", "f64"):
        t0 = time.perf_counter()
        sv = lowd.Solver(g.n, src, dst, w, state, star_max=16)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        print(f"[bench] {state} setup {t_setup:.1f}s info {sv.info()}", flush=True)
        r = timed_single(sv, g.m, args, stream, torch, state)
        r["setup_s"] = t_setup
        r["info"] = sv.info()
        res[state] = (r, sv)
        if state == "f32k":
            # loads after the FP32 run's sweep count, for the error against FP64
            sv.reset(stream)
            sv.iterate(r["last_sweeps"], stream)
            _, L32 = sv.read_state(stream)
            res["L32"] = L32.cpu().numpy()
            sv.close()
    r64, sv64 = res["f64"]
    r32 = res["f32k"][0]
    sv64.reset(stream)
    sv64.iterate(r32["last_sweeps"], stream)
    _, L64 = sv64.read_state(stream)
    L64 = L64.cpu().numpy()
    err = float(np.max(np.abs(res["L32"] - L64)) / np.max(np.abs(L64)))
    sv64.close()
    out = base_line(args, r32["value"], r32["elapsed"] / args.steps * 1e3, "f32k",
                    {"workload": g.name + " (" + WORKLOADS["chunglu4m"] + "), FP32 fractions + "
                     "compensated FP32 loads vs FP64, to 1e-6 gap", "n": g.n, "m": g.m,
                     "star_max": 16, "check_every": args.check_every, "seed": args.seed})
    out.update({
        "time_to_1e-6_ms": r32["elapsed"] / args.steps * 1e3,
        "sweeps_to_1e-6": r32["last_sweeps"],
        "density": density_str(r32["ex"], True),
        "sweep_ms": r32["per_sweep_s"] * 1e3,
        "setup_s": r32["setup_s"],
        "schedule": r32["info"],
        "roofline": roofline(sweep_bytes(g.n, g.m, 4, 4, 8), r32["per_sweep_s"],
                             "one FP32 sweep (HIP graph)"),
        "f64": {"value": r64["value"], "time_to_1e-6_ms": r64["elapsed"] / args.steps * 1e3,
                "sweeps_to_1e-6": r64["last_sweeps"], "density": density_str(r64["ex"], True),
                "sweep_ms": r64["per_sweep_s"] * 1e3,
                "roofline": roofline(sweep_bytes(g.n, g.m, 8, 4, 8), r64["per_sweep_s"],
                                     "one FP64 sweep (HIP graph)")},
        "f32k_load_error_vs_f64": {"max_abs_over_max": err, "sweeps": r32["last_sweeps"],
                                   "note": "FP64 path is bit-identical to the FP64 oracle"},
    })
    return out


def run_rmat24(args, torch, lowd, synth):
    t0 = time.perf_counter()
    g = synth.workload(3, seed=args.seed)
    print(f"[bench] workload {g.name}: n={g.n} m={g.m} generated in "
          f"{time.perf_counter() - t0:.1f}s", flush=True)
    src = torch.from_numpy(g.src).cuda()
    dst = torch.from_numpy(g.dst).cuda()
    stream = torch.cuda.current_stream()
    pr = lowd.prune(g.n, src, dst, stream)          # warm-up (allocations, code load)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pr = lowd.prune(g.n, src, dst, stream)
    torch.cuda.synchronize()
    t_prune = time.perf_counter() - t0
    print(f"[bench] prune {t_prune * 1e3:.1f} ms: rounds {pr['rounds']} H n={pr['n_h']} "
          f"m={pr['m_h']}", flush=True)
    hs = pr["src"].clone()
    hd = pr["dst"].clone()
    state = args.state or "f32k"
    t0 = time.perf_counter()
    sv = lowd.Solver(pr["n_h"], hs, hd, None, state, star_max=16)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    print(f"[bench] setup {t_setup:.1f}s info {sv.info()}", flush=True)
    r = timed_single(sv, pr["m_h"], args, stream, torch, state)
    xb = 4 if state == "f32k" else 8
    out = base_line(args, r["value"], r["elapsed"] / args.steps * 1e3 + t_prune * 1e3, state,
                    {"workload": g.name + " (" + WORKLOADS["rmat24"] + "), then LOWD on H in " +
                     state.upper() + ", to 1e-6 gap", "n": g.n, "m": g.m, "n_h": pr["n_h"],
                     "m_h": pr["m_h"], "star_max": 16, "check_every": args.check_every,
                     "seed": args.seed})
    out.update({
        "prune_ms": t_prune * 1e3,
        "prune_rounds": pr["rounds"],
        "prune_edges_per_s": g.m / t_prune,
        "time_to_1e-6_ms": r["elapsed"] / args.steps * 1e3,
        "sweeps_to_1e-6": r["last_sweeps"],
        "density": density_str(r["ex"]),
        "sweep_ms": r["per_sweep_s"] * 1e3,
        "setup_s": t_setup,
        "schedule": sv.info(),
        "roofline": roofline(sweep_bytes(pr["n_h"], pr["m_h"], xb, 0, 8), r["per_sweep_s"],
                             "one sweep of H (HIP graph)"),
    })
    sv.close()
    # Algorithm 2's other plug-in: greedy peeling (Algorithm 3) of H
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gr = lowd.greedy_peel(pr["n_h"], hs, hd, stream)
    torch.cuda.synchronize()
    t_greedy = time.perf_counter() - t0
    out["greedy_on_h"] = {"ms": t_greedy * 1e3, "density": f"{gr['num']}/{gr['den']}",
                          "vs_lowd_density": (gr["num"] / gr["den"]) /
                                             (r["ex"]["num"] / r["ex"]["den"])}
    print(f"[bench] greedy on H: {t_greedy * 1e3:.1f} ms, density {gr['num']}/{gr['den']}",
          flush=True)
    return out


def run_uniform(args, torch, lowd, synth):
    """The sweep where phases are wide: a uniform random graph has a small
    maximum degree, so a sweep is a few dozen phases of millions of edges
    each, and the kernels run at memory speed.  Times sweeps only."""
    t0 = time.perf_counter()
    g = synth.uniform_pairs(25, 28, seed=args.seed)
    print(f"[bench] workload {g.name}: n={g.n} m={g.m} generated in "
          f"{time.perf_counter() - t0:.1f}s", flush=True)
    src = torch.from_numpy(g.src).cuda()
    dst = torch.from_numpy(g.dst).cuda()
    del g.src, g.dst
    stream = torch.cuda.current_stream()
    state = args.state or "f32k"
    t0 = time.perf_counter()
    sv = lowd.Solver(g.n, src, dst, None, state, star_max=16)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    info = sv.info()
    print(f"[bench] setup {t_setup:.1f}s info {info}", flush=True)
    ev_a = torch.cuda.Event(enable_timing=True)
    ev_b = torch.cuda.Event(enable_timing=True)
    sv.iterate(max(args.warmup, 1), stream)
    sweeps = 10 * args.steps
    ev_a.record(stream)
    sv.iterate(sweeps, stream)
    ev_b.record(stream)
    ev_b.synchronize()
    per = ev_a.elapsed_time(ev_b) / 1e3 / sweeps
    m = info["m"]
    xb = 4 if state == "f32k" else 8
    out = base_line(args, m / per, per * 1e3, state,
                    {"workload": WORKLOADS["uniform"], "n": g.n, "m": m, "star_max": 16,
                     "seed": args.seed})
    out.update({"sweep_ms": per * 1e3, "sweeps_timed": sweeps, "setup_s": t_setup,
                "schedule": info,
                "roofline": roofline(sweep_bytes(g.n, m, xb, 0, 8), per,
                                     "one sweep (HIP graph); wide phases")})
    sv.close()
    return out


def batch_solves(gs, state, args, torch, lowd, stream):
    """Prepares (and tunes) the batch in one state, then times args.steps
    solves after args.warmup untimed ones.  Each solve: reset; then sweep the
    graphs still above the tolerance, k sweeps a launch, extract and retire,
    until every graph is within it.  Once fewer than an eighth of the graphs
    remain, k doubles after each check, up to 8 K (FP64) or 4 K (FP32K): the
    few slow graphs then cost a check more than a sweep, but a longer launch
    overshoots their convergence, and for FP32K lets the carried loads drift
    further from the fractions' loads between two restarts."""
    M = sum(g.m for g in gs)
    t0 = time.perf_counter()
    b = lowd.Batch(gs, state, tune=True, stream=stream)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    info = b.info()
    print(f"[bench] {state} prepare + tune {t_setup:.1f}s info {info}", flush=True)
    ev_a = torch.cuda.Event(enable_timing=True)
    ev_b = torch.cuda.Event(enable_timing=True)
    K = args.check_every

    def one_solve():
        b.reset(stream)
        updates, launches, sweeps, launch_s, launch_bytes = 0, 0, 0, 0.0, 0
        active, aedges = len(gs), M
        k = K
        while active > 0:
            if active * 8 < len(gs):
                k = min(2 * k, (4 if state == "f32k" else 8) * K)
            ev_a.record(stream)
            b.iterate(k, stream)
            ev_b.record(stream)
            b.extract(stream)
            ev_b.synchronize()
            launch_s += ev_a.elapsed_time(ev_b) / 1e3
            updates += aedges * k
            launch_bytes += aedges * k * (8 + 2 * (4 if state == "f32k" else 8))
            launches += 1
            sweeps += k
            active, aedges = b.retire(args.tol, stream)
            if sweeps > 20000:
                raise RuntimeError("no convergence within 20000 sweeps")
        return updates, launches, sweeps, launch_s, launch_bytes

    for i in range(args.warmup):
        u, l, s_, _, _ = one_solve()
        print(f"[bench] {state} warmup {i}: {s_} sweeps in {l} launches, {u} edge updates",
              flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = dict(updates=0, launches=0, launch_s=0.0, bytes=0, last=None, setup_s=t_setup, info=info)
    for i in range(args.steps):
        u, l, s_, ls, lb = one_solve()
        r["updates"] += u
        r["launches"] += l
        r["launch_s"] += ls
        r["bytes"] += lb
        r["last"] = (u, l, s_)
        print(f"[bench] {state} step {i}: {s_} sweeps in {l} launches", flush=True)
    torch.cuda.synchronize()
    r["elapsed"] = time.perf_counter() - t0
    b.extract(stream)
    r["gaps"] = b.gaps()
    r["num"] = b.num.cpu().numpy()
    r["den"] = b.den.cpu().numpy()
    b.close()
    return r


def run_batch4096(args, torch, lowd, synth):
    t0 = time.perf_counter()
    gs = synth.workload(4, seed=args.seed)
    M = sum(g.m for g in gs)
    N = sum(g.n for g in gs)
    print(f"[bench] {len(gs)} graphs, N={N} M={M}, generated in {time.perf_counter() - t0:.1f}s",
          flush=True)
    state = args.state or "f32k"
    stream = torch.cuda.current_stream()
    r = batch_solves(gs, state, args, torch, lowd, stream)
    last = r["last"]
    out = base_line(args, r["updates"] / r["elapsed"], r["elapsed"] / args.steps * 1e3, state,
                    {"workload": WORKLOADS["batch4096"] + ", " + state.upper() +
                     ", every graph to a 1e-6 gap, converged graphs retired",
                     "graphs": len(gs), "N": N, "M": M, "star_max": 16,
                     "check_every": args.check_every, "seed": args.seed})
    out.update({
        "time_to_1e-6_ms": r["elapsed"] / args.steps * 1e3,
        "sweeps_to_1e-6": last[2],
        "launches": last[1],
        "edge_updates_per_solve": last[0],
        "max_gap": float(np.max(r["gaps"])),
        "densities_sum": f"{int(r['num'].sum())}/{int(r['den'].sum())}",
        "setup_s": r["setup_s"],
        "batch": r["info"],
        "roofline": roofline(r["bytes"] / max(r["launches"], 1),
                             r["launch_s"] / max(r["launches"], 1),
                             "one persistent launch of k sweeps over the graphs still "
                             "iterating (LDS-resident; HBM carries ids, fractions and the "
                             "loads in and out)"),
    })
    # the same batch in the other state, for comparison
    other = "f64" if state == "f32k" else "f32k"
    r2 = batch_solves(gs, other, args, torch, lowd, stream)
    out[other] = {"time_to_1e-6_ms": r2["elapsed"] / args.steps * 1e3,
                  "sweeps_to_1e-6": r2["last"][2], "launches": r2["last"][1],
                  "max_gap": float(np.max(r2["gaps"])),
                  "densities_sum": f"{int(r2['num'].sum())}/{int(r2['den'].sum())}"}
    if args.per_graph_sample > 0:
        out["per_graph_f64"] = per_graph_baseline(gs, args, torch, lowd, stream)
    return out


def per_graph_baseline(gs, args, torch, lowd, stream):
    """The plain FP64 per-graph form on a sample: every k-th graph of the
    batch (in size order, so the sample spans the sizes) solved on its own
    with the single-graph solver to the same gap; scaled to the batch."""
    order = sorted(range(len(gs)), key=lambda i: -gs[i].m)
    step = max(1, len(gs) // args.per_graph_sample)
    sample = order[::step]
    ev_a = torch.cuda.Event(enable_timing=True)
    ev_b = torch.cuda.Event(enable_timing=True)
    t_setup = t_solve = 0.0
    for i in sample:
        g = gs[i]
        t0 = time.perf_counter()
        sv = lowd.Solver(g.n, torch.from_numpy(g.src).cuda(), torch.from_numpy(g.dst).cuda(),
                         None, "f64", star_max=16)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        single_solve(sv, stream, args.tol, args.check_every, ev_a, ev_b)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        t_setup += t1 - t0
        t_solve += t2 - t1
        sv.close()
    scale = len(gs) / len(sample)
    return {"sample_graphs": len(sample), "scaled_solve_ms": t_solve * scale * 1e3,
            "scaled_setup_ms": t_setup * scale * 1e3,
            "note": "each graph solved alone (FP64 single-graph solver, same 1e-6 gap); "
                    "sample times scaled by graphs/sample"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--check-every", type=int, default=10)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="chunglu1m")
    ap.add_argument("--state", choices=["f64", "f32k"], default=None,
                    help="solver state (default: f64 for chunglu1m, f32k otherwise)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--per-graph-sample", type=int, default=64,
                    help="batch4096: graphs solved one by one in FP64 for comparison (0: none)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one plain device-to-device copy of this many MiB (a "
                         "known-size kernel for scaling memory counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the workload is one graph on one MI355X)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2307_15969_amd as lowd
    import synth

    torch.cuda.set_device(0)
    if args.copy_calibration_mib > 0:
        nbytes = args.copy_calibration_mib << 20
        a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: one copy of {nbytes} bytes", flush=True)
        del a, b
    run = {"chunglu1m": run_chunglu1m, "chunglu4m": run_chunglu4m, "rmat24": run_rmat24,
           "batch4096": run_batch4096, "uniform": run_uniform}[args.workload]
    out = run(args, torch, lowd, synth)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
