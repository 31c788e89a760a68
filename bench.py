"""Benchmark: LOWD on the Chung-Lu power-law workload (n = 1M nodes, ~10M
unit-weight edges, degree exponent 2.1, a planted 500-node block of pair
density 0.3), FP64 state, no pruning, solved to a 1e-6 relative density
gap.

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

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PROFILE = os.path.join(ROOT, "profiles", "sweep_chunglu_1M_10M_f64.md")
SWEEP_SOURCES = ["paper_2307_15969_amd/csrc/k_sweep.hip", "paper_2307_15969_amd/csrc/sweep_state.h",
                 "paper_2307_15969_amd/csrc/schedule.cpp", "paper_2307_15969_amd/csrc/lowd_internal.h",
                 "paper_2307_15969_amd/csrc/api.hip"]


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--check-every", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run one plain device-to-device copy of this many MiB (a "
                         "known-size kernel for scaling memory counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the workload is one graph on one MI355X)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
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
    t0 = time.perf_counter()
    g = synth.workload(1, seed=args.seed)
    t_gen = time.perf_counter() - t0
    print(f"[bench] workload {g.name}: n={g.n} m={g.m} generated in {t_gen:.1f}s", flush=True)
    src = torch.from_numpy(g.src).cuda()
    dst = torch.from_numpy(g.dst).cuda()
    stream = torch.cuda.current_stream()
    t0 = time.perf_counter()
    sv = lowd.Solver(g.n, src, dst, None, "f64", star_max=16)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    info = sv.info()
    print(f"[bench] setup (validation, schedule, CSR, init) {t_setup:.2f}s info {info}",
          flush=True)

    ev_a = torch.cuda.Event(enable_timing=True)
    ev_b = torch.cuda.Event(enable_timing=True)

    def one_solve(record):
        """reset, then sweep/check until the gap tolerance; returns
        (sweeps, sweep seconds measured with events, final extraction)."""
        sv.reset(stream)
        sweeps = 0
        sweep_s = 0.0
        ex = sv.extract(stream)
        while ex["gap"] > args.tol:
            ev_a.record(stream)
            sv.iterate(args.check_every, stream)
            ev_b.record(stream)
            ev_b.synchronize()
            sweep_s += ev_a.elapsed_time(ev_b) / 1e3
            sweeps += args.check_every
            ex = sv.extract(stream)
            if sweeps > 20000:
                raise RuntimeError("no convergence within 20000 sweeps")
        return sweeps, sweep_s, ex

    for i in range(args.warmup):
        s, ss, ex = one_solve(False)
        print(f"[bench] warmup {i}: {s} sweeps, gap {ex['gap']:.3e}, "
              f"density {ex['num']}/{ex['den']}", flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tot_sweeps = 0
    tot_sweep_s = 0.0
    results = []
    for i in range(args.steps):
        s, ss, ex = one_solve(True)
        tot_sweeps += s
        tot_sweep_s += ss
        results.append((s, ex["num"], ex["den"], ex["gap"]))
        print(f"[bench] step {i}: {s} sweeps, gap {ex['gap']:.3e}", flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    ms_per_step = elapsed / args.steps * 1e3
    value = g.m * tot_sweeps / elapsed
    per_sweep_s = tot_sweep_s / max(tot_sweeps, 1)
    bytes_sweep = sweep_bytes(g.n, g.m)
    achieved = bytes_sweep / per_sweep_s / 1e9
    out = {
        "metric": "LOWD edge-updates/s + % HBM roofline; time to density within 1e-6 of optimum",
        "value": value,
        "unit": "edge-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": g.name + " (Chung-Lu n=1M, ~10M unit edges, beta 2.1, planted "
                               "500-node block p=0.3), FP64, no pruning, to 1e-6 gap",
                   "n": g.n, "m": g.m, "star_max": 16, "check_every": args.check_every,
                   "seed": args.seed},
        "time_to_1e-6_ms": ms_per_step,
        "sweeps_to_1e-6": results[-1][0],
        "density": f"{results[-1][1]}/{results[-1][2]}",
        "sweep_ms": per_sweep_s * 1e3,
        "sweep_edge_updates_per_s": g.m / per_sweep_s,
        "setup_s": t_setup,
        "schedule": info,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": profiled_traffic(),
                     "kernel": "one sweep (the HIP graph of phase kernels + LDS tail kernel)",
                     "algorithmic_bytes": bytes_sweep},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
