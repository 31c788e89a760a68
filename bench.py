"""Benchmark: LOWD on R-MAT scale 24 (16.8M nodes, edge factor 16, quadrant
probabilities .57/.19/.19/.05, ~260M unit edges after symmetrising and
de-duplication), pruned by Algorithm 2, then solved on the pruned graph H to a
1e-6 relative density gap: FP64 in `value`, the FP32 + compensated-load state
beside it.  Other workloads (--workload): chunglu1m (1M nodes, ~10M unit
edges, FP64, no pruning), chunglu4m (4M nodes, ~64M lognormal edges, FP32K
against FP64), batch4096 (4096 small graphs in the batched form) and uniform
(a wide-phase diagnostic of the sweep, not a paper workload).

One step = the hot path once, on inputs resident in HBM: Algorithm 2's prune
of G (where the workload prunes), then a solve of H from Algorithm 1's
initial state (reset of fractions and loads, sweeps, checks with the dual
bound D and the extraction) through lowd_solve until (D - rho) / rho <= 1e-6.
The phase schedule is built once per graph, before timing (setup_s).

Printed: one JSON line.  `value` is edge updates of the solves (|E(H)| x
sweeps) per second of solve; `roofline` is the sweep's algorithmic bytes over
its time, measured with HIP events on the stream the sweeps run on;
`cpu_baseline` is the CPU oracle's edge loop timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# the sources that decide the sweep's kernels and memory layout; a committed
# counter summary is used only while they are unchanged
SWEEP_SOURCES = ["paper_2307_15969_amd/csrc/k_sweep.hip", "paper_2307_15969_amd/csrc/sweep_state.h",
                 "paper_2307_15969_amd/csrc/schedule.cpp", "paper_2307_15969_amd/csrc/lowd_internal.h"]
PROFILES = {
    "rmat24": os.path.join(ROOT, "profiles", "sweep_rmat24_H_f64.md"),
    "chunglu1m": os.path.join(ROOT, "profiles", "sweep_chunglu_1M_10M_f64.md"),
    "uniform": os.path.join(ROOT, "profiles", "sweep_uniform_f64.md"),
}


def sources_hash() -> str:
    h = hashlib.sha256()
    for p in SWEEP_SOURCES:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def profiled_traffic(workload: str):
    """HBM bytes per sweep from the committed FETCH_SIZE/WRITE_SIZE summary of
    this workload's FP64 sweep, or None when the sweep sources changed since
    the counters were taken (the summary records a hash of those sources)."""
    try:
        text = open(PROFILES[workload]).read()
    except (OSError, KeyError):
        return None
    fields = dict(l.split(": ", 1) for l in text.splitlines()
                  if l.startswith(("traffic_bytes_per_sweep: ", "sources_sha256_16: ")))
    if fields.get("sources_sha256_16", "").strip() != sources_hash():
        return None
    if "traffic_bytes_per_sweep" not in fields:
        return None
    return int(fields["traffic_bytes_per_sweep"])


def sweep_bytes(n: int, m: int, x_bytes: int = 8, w_bytes: int = 0, l_bytes: int = 8) -> int:
    """Algorithmic bytes of one sweep: every edge reads its two endpoint ids
    (8 B), reads and writes its fraction, reads its weight; every node's load
    is read and written once."""
    return m * (8 + 2 * x_bytes + w_bytes) + n * 2 * l_bytes


def cpu_baseline(n, src, dst, w, seconds: float = 12.0) -> dict:
    """The FP64 oracle (sequential, one core): initialisation, then full
    passes of Algorithm 1's edge loop in edge-index order over the same
    graph, for about `seconds`."""
    import oracle
    oracle.build(force=False)
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    m = src.size
    order = np.arange(m, dtype=np.int32)
    x, L = oracle.init(n, src, dst, w)
    sweeps = 0
    t0 = time.perf_counter()
    while True:
        oracle.sweep(n, src, dst, w, order, 1, x, L)
        sweeps += 1
        el = time.perf_counter() - t0
        if el >= seconds or sweeps >= 200:
            break
    return {"value": m * sweeps / el, "unit": "edge-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{sweeps} full passes of the edge loop over the same {m}-edge graph, "
                      f"edge-index order ({el:.1f} s)",
            "sweep_s": el / sweeps, "host": host_cpu()}


def host_cpu() -> str:
    """The host's CPU model and logical core count (for the CPU baseline)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return f"{model}, {os.cpu_count()} logical cores"


WORKLOADS = {
    "rmat24": "R-MAT scale 24, edge factor 16, (.57,.19,.19,.05), pruned by Algorithm 2, "
              "then LOWD on H",
    "chunglu1m": "Chung-Lu n=1M, ~10M unit edges, beta 2.1, planted 500-node block p=0.3",
    "chunglu4m": "Chung-Lu n=4M, ~64M lognormal(0,1) edges (float32), beta 2.1, planted block",
    "batch4096": "4096 Chung-Lu graphs (beta 2.3), edges log-uniform in [100, 50000], "
                 "planted blocks of 5-40 nodes",
    "uniform": "diagnostic: uniform random pairs (few wide phases); sweeps only",
}


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


def density_str(r, weighted=False):
    """the extracted density: the exact rational for unit weights, else the
    FP64 weight sum over the node count"""
    if weighted:
        return f"{r['num_w']!r}/{r['den']}"
    return f"{r['num']}/{r['den']}"


def one_solve(sv, args, stream):
    sv.reset(stream)
    r = sv.solve(args.tol, args.max_sweeps, args.check_every, stream)
    if not r["converged"]:
        raise RuntimeError(f"no convergence within {args.max_sweeps} sweeps (gap {r['gap']:.3e})")
    return r


def sweep_seconds(sv, sweeps, stream, torch):
    """Average time of one sweep: `sweeps` replays of the sweep's HIP graph
    from the initial state, timed with events on the stream they run on."""
    ev_a = torch.cuda.Event(enable_timing=True)
    ev_b = torch.cuda.Event(enable_timing=True)
    sv.reset(stream)
    sv.iterate(1, stream)
    sv.reset(stream)
    ev_a.record(stream)
    sv.iterate(sweeps, stream)
    ev_b.record(stream)
    ev_b.synchronize()
    return ev_a.elapsed_time(ev_b) / 1e3 / sweeps


def timed_solves(sv, m, args, stream, torch, label, before_each=None):
    """args.warmup untimed solves, then args.steps timed ones (each from the
    initial state); before_each() runs inside the timed region first (the
    prune, where the workload prunes) and returns its seconds."""
    for i in range(args.warmup):
        if before_each:
            before_each()
        r = one_solve(sv, args, stream)
        print(f"[bench] {label} warmup {i}: {r['sweeps']} sweeps, gap {r['gap']:.3e}, "
              f"density {r['num']}/{r['den']}", flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot_sweeps, solve_s, pre_s, last = 0, 0.0, 0.0, None
    for i in range(args.steps):
        if before_each:
            pre_s += before_each()
        ta = time.perf_counter()
        r = one_solve(sv, args, stream)
        solve_s += time.perf_counter() - ta
        tot_sweeps += r["sweeps"]
        last = r
        print(f"[bench] {label} step {i}: {r['sweeps']} sweeps, gap {r['gap']:.3e}", flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    per_sweep = sweep_seconds(sv, max(last["sweeps"], 1), stream, torch)
    return dict(elapsed=elapsed, sweeps=tot_sweeps, solve_s=solve_s, pre_s=pre_s, last=last,
                value=m * tot_sweeps / solve_s, per_sweep_s=per_sweep)


def state_result(r, m, n, xb, wb, kernel, traffic=None, weighted=False):
    return {"value": r["value"], "time_to_1e-6_ms": r["solve_s"] / max(len_steps(r), 1) * 1e3,
            "sweeps_to_1e-6": r["last"]["sweeps"], "density": density_str(r["last"], weighted),
            "gap": r["last"]["gap"], "sweep_ms": r["per_sweep_s"] * 1e3,
            "sweep_edge_updates_per_s": m / r["per_sweep_s"],
            "roofline": roofline(sweep_bytes(n, m, xb, wb, 8), r["per_sweep_s"], kernel, traffic)}


def len_steps(r):
    return r.get("steps", 1)


def load_error(sv_a, sv_b, sweeps, stream):
    """max |L_a - L_b| / max |L_b| after the same number of sweeps from the
    initial state"""
    sv_a.reset(stream)
    sv_a.iterate(sweeps, stream)
    _, La = sv_a.read_state(stream)
    sv_b.reset(stream)
    sv_b.iterate(sweeps, stream)
    _, Lb = sv_b.read_state(stream)
    La, Lb = La.cpu().numpy(), Lb.cpu().numpy()
    return float(np.max(np.abs(La - Lb)) / np.max(np.abs(Lb)))


def run_rmat24(args, torch, lowd, synth):
    t0 = time.perf_counter()
    g = synth.rmat(24, 16, seed=args.seed, device="cuda")
    print(f"[bench] workload {g.name}: n={g.n} m={g.m} generated in "
          f"{time.perf_counter() - t0:.1f}s", flush=True)
    src = torch.from_numpy(g.src).cuda()
    dst = torch.from_numpy(g.dst).cuda()
    n, m = g.n, g.m
    del g
    stream = torch.cuda.current_stream()
    pr = lowd.prune(n, src, dst, stream)          # warm-up (allocations, code load)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pr = lowd.prune(n, src, dst, stream)
    torch.cuda.synchronize()
    t_prune = time.perf_counter() - t0
    n_h, m_h = pr["n_h"], pr["m_h"]
    print(f"[bench] prune {t_prune * 1e3:.1f} ms: rounds {pr['rounds']} H n={n_h} m={m_h}",
          flush=True)
    hs = pr["src"].clone()
    hd = pr["dst"].clone()
    del pr

    def prune_again():
        torch.cuda.synchronize()
        ta = time.perf_counter()
        lowd.prune(n, src, dst, stream)
        torch.cuda.synchronize()
        return time.perf_counter() - ta

    res, svs = {}, {}
    for state in ((args.state,) if args.state else ("f64", "f32k")):
        t0 = time.perf_counter()
        sv = lowd.Solver(n_h, hs, hd, None, state, star_max=args.star_max)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        print(f"[bench] {state} setup {t_setup:.1f}s info {sv.info()}", flush=True)
        r = timed_solves(sv, m_h, args, stream, torch, state, prune_again)
        r["steps"] = args.steps
        r["setup_s"] = t_setup
        res[state] = r
        svs[state] = sv
    lead = "f64" if "f64" in res else "f32k"
    r64, r32 = res[lead], res.get("f32k")
    err = (load_error(svs["f32k"], svs["f64"], r32["last"]["sweeps"], stream)
           if len(res) == 2 else None)
    info = svs[lead].info()
    for sv in svs.values():
        sv.close()
    step_ms = (r64["pre_s"] + r64["solve_s"]) / args.steps * 1e3
    name = {"f64": "FP64", "f32k": "FP32K"}[lead]
    out = base_line(args, r64["value"], step_ms, lead,
                    {"workload": f"rmat24 ({WORKLOADS['rmat24']}), {name} to a 1e-6 gap; "
                     "step = prune + solve", "n": n, "m": m, "n_h": n_h, "m_h": m_h,
                     "star_max": args.star_max, "check_every": args.check_every,
                     "seed": args.seed})
    f64 = state_result(r64, m_h, n_h, 8 if lead == "f64" else 4, 0,
                       f"one {name} sweep of H (HIP graph of phase kernels and "
                       "single-workgroup tiers)",
                       profiled_traffic("rmat24") if lead == "f64" else None)
    out.update({
        "prune_ms": t_prune * 1e3,
        "prune_edges_per_s": m / t_prune,
        "time_to_1e-6_ms": step_ms,
        "solve_ms": f64["time_to_1e-6_ms"],
        "sweeps_to_1e-6": f64["sweeps_to_1e-6"],
        "density": f64["density"],
        "sweep_ms": f64["sweep_ms"],
        "setup_s": r64["setup_s"],
        # once, from G: prune, then the solver's setup on H (schedule and
        # layout), then the solve
        "total_with_setup_ms": t_prune * 1e3 + r64["setup_s"] * 1e3 + f64["time_to_1e-6_ms"],
        "schedule": info,
        "roofline": f64["roofline"],
    })
    if err is not None:
        f32 = state_result(r32, m_h, n_h, 4, 0, "one FP32K sweep of H (HIP graph)")
        out.update({
            "f32k": dict(f32, setup_s=r32["setup_s"],
                         step_ms=(r32["pre_s"] + r32["solve_s"]) / args.steps * 1e3),
            "f32k_load_error_vs_f64": {"max_abs_over_max": err, "sweeps": r32["last"]["sweeps"]},
        })
    if not args.no_cpu_baseline:
        torch.cuda.synchronize()
        h_src, h_dst = hs.cpu().numpy(), hd.cpu().numpy()
        out["cpu_baseline"] = cpu_baseline(n_h, h_src, h_dst, None, args.cpu_seconds)
        out["cpu_baseline"]["sample"] += " (the pruned graph H)"
        # as many oracle passes as the GPU solve made sweeps
        out["cpu_baseline"]["solve_sweeps_s"] = (out["cpu_baseline"]["sweep_s"] *
                                                f64["sweeps_to_1e-6"])
    return out


def run_chunglu1m(args, torch, lowd, synth):
    t0 = time.perf_counter()
    g = synth.workload(1, seed=args.seed)
    print(f"[bench] workload {g.name}: n={g.n} m={g.m} generated in "
          f"{time.perf_counter() - t0:.1f}s", flush=True)
    src = torch.from_numpy(g.src).cuda()
    dst = torch.from_numpy(g.dst).cuda()
    stream = torch.cuda.current_stream()
    state = args.state or "f64"
    t0 = time.perf_counter()
    sv = lowd.Solver(g.n, src, dst, None, state, star_max=args.star_max)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    info = sv.info()
    print(f"[bench] setup {t_setup:.2f}s info {info}", flush=True)
    r = timed_solves(sv, g.m, args, stream, torch, state)
    r["steps"] = args.steps
    sv.close()
    xb = 8 if state == "f64" else 4
    res = state_result(r, g.m, g.n, xb, 0, "one sweep (HIP graph of phase kernels and "
                       "single-workgroup tiers)",
                       profiled_traffic("chunglu1m") if state == "f64" else None)
    out = base_line(args, r["value"], r["solve_s"] / args.steps * 1e3, state,
                    {"workload": f"{g.name} ({WORKLOADS['chunglu1m']}), {state.upper()}, "
                     "no pruning, to a 1e-6 gap", "n": g.n, "m": g.m,
                     "star_max": args.star_max, "check_every": args.check_every,
                     "seed": args.seed})
    out.update(res)
    out.update({"setup_s": t_setup, "schedule": info})
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g.n, g.src, g.dst, None, args.cpu_seconds)
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
    res, svs = {}, {}
    for state in ("f32k", "f64"):
        t0 = time.perf_counter()
        sv = lowd.Solver(g.n, src, dst, w, state, star_max=args.star_max)
        torch.cuda.synchronize()
        t_setup = time.perf_counter() - t0
        print(f"[bench] {state} setup {t_setup:.1f}s info {sv.info()}", flush=True)
        r = timed_solves(sv, g.m, args, stream, torch, state)
        r["steps"] = args.steps
        r["setup_s"] = t_setup
        res[state] = r
        svs[state] = sv
    r32, r64 = res["f32k"], res["f64"]
    err = load_error(svs["f32k"], svs["f64"], r32["last"]["sweeps"], stream)
    info = svs["f32k"].info()
    for sv in svs.values():
        sv.close()
    f32 = state_result(r32, g.m, g.n, 4, 4, "one FP32K sweep (HIP graph)", None, True)
    f64 = state_result(r64, g.m, g.n, 8, 4, "one FP64 sweep (HIP graph)", None, True)
    out = base_line(args, r32["value"], r32["solve_s"] / args.steps * 1e3, "f32k",
                    {"workload": f"{g.name} ({WORKLOADS['chunglu4m']}), FP32 fractions + "
                     "compensated loads vs FP64, to a 1e-6 gap", "n": g.n, "m": g.m,
                     "star_max": args.star_max, "check_every": args.check_every,
                     "seed": args.seed})
    out.update(f32)
    out.update({"setup_s": r32["setup_s"], "schedule": info, "f64": f64,
                "f32k_load_error_vs_f64": {"max_abs_over_max": err,
                                           "sweeps": r32["last"]["sweeps"],
                                           "note": "the FP64 path is bit-identical to the FP64 "
                                                   "oracle"}})
    return out


def run_uniform(args, torch, lowd, synth):
    """The sweep where phases are wide: a uniform random graph has a small
    maximum degree, so a sweep is a few dozen phases of millions of edges
    each, and bytes, not phase latency, bound it.  Times sweeps only."""
    t0 = time.perf_counter()
    g = synth.uniform_pairs(args.uniform_log_n, args.uniform_log_m, seed=args.seed,
                            device="cuda")
    print(f"[bench] workload {g.name}: n={g.n} m={g.m} generated in "
          f"{time.perf_counter() - t0:.1f}s", flush=True)
    src = torch.from_numpy(g.src).cuda()
    dst = torch.from_numpy(g.dst).cuda()
    n, m = g.n, g.m
    del g
    stream = torch.cuda.current_stream()
    state = args.state or "f64"
    t0 = time.perf_counter()
    sv = lowd.Solver(n, src, dst, None, state, star_max=args.star_max)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    info = sv.info()
    print(f"[bench] setup {t_setup:.1f}s info {info}", flush=True)
    sweeps = 10 * args.steps
    per = sweep_seconds(sv, sweeps, stream, torch)
    sv.close()
    xb = 4 if state == "f32k" else 8
    out = base_line(args, m / per, per * 1e3, state,
                    {"workload": f"{WORKLOADS['uniform']}: 2^{args.uniform_log_m} pairs on "
                     f"2^{args.uniform_log_n} nodes", "n": n, "m": m,
                     "star_max": args.star_max, "seed": args.seed})
    out.update({"sweep_ms": per * 1e3, "sweeps_timed": sweeps, "setup_s": t_setup,
                "schedule": info,
                "roofline": roofline(sweep_bytes(n, m, xb, 0, 8), per,
                                     "one sweep (HIP graph); wide phases",
                                     profiled_traffic("uniform") if state == "f64" else None)})
    return out


def batch_solves(gs, state, args, torch, lowd, stream):
    """Prepares (and tunes) the batch in one state, then times args.steps
    solves after args.warmup untimed ones; each solve: reset, then
    lowd_batch_solve_prepared to the tolerance."""
    t0 = time.perf_counter()
    b = lowd.Batch(gs, state, tune=True, stream=stream)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    info = b.info()
    print(f"[bench] {state} prepare + tune {t_setup:.1f}s info {info}", flush=True)
    m = np.array([g.m for g in gs], dtype=np.int64)

    def one():
        b.reset(stream)
        r = b.solve(args.tol, args.max_sweeps, args.check_every, stream)
        if not r["converged"]:
            raise RuntimeError(f"batch: no convergence within {args.max_sweeps} sweeps")
        return r

    for i in range(args.warmup):
        r = one()
        print(f"[bench] {state} warmup {i}: most sweeps {int(r['sweeps'].max())}", flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    updates = 0
    for i in range(args.steps):
        r = one()
        updates += int((m * r["sweeps"]).sum())
        print(f"[bench] {state} step {i}: most sweeps {int(r['sweeps'].max())}", flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    num, den, D = b.num.cpu().numpy(), b.den.cpu().numpy(), b.D.cpu().numpy()
    rho = num / np.maximum(den, 1)
    with np.errstate(divide="ignore", invalid="ignore"):
        gaps = np.where(rho > 0, (D - rho) / rho, 0.0)
    b.close()
    return dict(elapsed=elapsed, updates=updates, sweeps=r["sweeps"], setup_s=t_setup, info=info,
                max_gap=float(np.max(gaps)), num=num, den=den)


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
    per_solve = r["elapsed"] / args.steps
    xb = 4 if state == "f32k" else 8
    out = base_line(args, r["updates"] / r["elapsed"], per_solve * 1e3, state,
                    {"workload": WORKLOADS["batch4096"] + ", " + state.upper() +
                     ", every graph to a 1e-6 gap", "graphs": len(gs), "N": N, "M": M,
                     "star_max": args.star_max, "check_every": args.check_every,
                     "seed": args.seed})
    m = np.array([g.m for g in gs], dtype=np.int64)
    n = np.array([g.n for g in gs], dtype=np.int64)
    bytes_solve = int((r["sweeps"] * (m * (8 + 2 * xb) + n * 16)).sum())
    out.update({
        "time_to_1e-6_ms": per_solve * 1e3,
        "most_sweeps": int(r["sweeps"].max()),
        "edge_updates_per_solve": r["updates"] // args.steps,
        "max_gap": r["max_gap"],
        "densities_sum": f"{int(r['num'].sum())}/{int(r['den'].sum())}",
        "setup_s": r["setup_s"],
        "batch": r["info"],
        "roofline": roofline(bytes_solve, per_solve,
                             "the whole batched solve (sweeps of every graph's schedule from LDS, "
                             "checks included); a loose model: the loads live in LDS"),
    })
    other = "f64" if state == "f32k" else "f32k"
    r2 = batch_solves(gs, other, args, torch, lowd, stream)
    out[other] = {"time_to_1e-6_ms": r2["elapsed"] / args.steps * 1e3,
                  "most_sweeps": int(r2["sweeps"].max()), "max_gap": r2["max_gap"],
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
    t_setup = t_solve = 0.0
    for i in sample:
        g = gs[i]
        t0 = time.perf_counter()
        sv = lowd.Solver(g.n, torch.from_numpy(g.src).cuda(), torch.from_numpy(g.dst).cuda(),
                         None, "f64", star_max=16)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        one_solve(sv, args, stream)
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
    ap.add_argument("--max-sweeps", type=int, default=20000)
    ap.add_argument("--star-max", type=int, default=None,
                    help="leaves per star per phase (default 32 for rmat24, whose pruned "
                         "graph's phase count a hub sets, else 16)")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="rmat24")
    ap.add_argument("--state", choices=["f64", "f32k"], default=None,
                    help="solver state: rmat24 runs only this one (default: FP64, then "
                         "FP32K beside it); chunglu1m: f64; batch4096 and uniform: the first "
                         "of two / the only one")
    ap.add_argument("--uniform-log-n", type=int, default=22)
    ap.add_argument("--uniform-log-m", type=int, default=28)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--per-graph-sample", type=int, default=64,
                    help="batch4096: graphs solved one by one in FP64 for comparison (0: none)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one plain device-to-device copy of this many MiB (a "
                         "known-size kernel for scaling memory counters)")
    args = ap.parse_args()
    if args.star_max is None:
        args.star_max = 32 if args.workload == "rmat24" else 16
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(every workload is sized for one MI355X)", file=sys.stderr)
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
