"""Writes chunglu4m.json: the oracle's results on the 4M-node Chung-Lu
workload with log-normal weights (about 63M edges), for the full-size GPU
test (tests/test_gpu_parity.py, test_chunglu4m_full_size_fp64_and_f32k).

Only the seeded input generator (synth) and the oracle run here: the
oracle's schedule with stars of at most 16 leaves, its initialisation and
22 sweeps (Algorithm 1; the benchmark's solve takes 22), then:
  - SHA-256 digests of the FP64 loads and fractions (the FP64 GPU path must
    match them bit for bit);
  - the loads of 4,096 nodes, exactly (as hexadecimal floats): the 2,048
    largest and 2,048 drawn with a fixed seed, for the FP32-compensated
    path's tolerance;
  - the maximum load D and the sum of the loads;
  - the densest prefix of the sorted loads: its edge count, its weight
    (the exact sum rounded once to FP64), its size and a digest of the set.
Run from the repository root:
    python tests/golden/make_chunglu4m.py
"""
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "..", ".."))

import oracle  # noqa: E402
import synth  # noqa: E402


def digest(a: np.ndarray) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def main() -> None:
    t0 = time.time()
    g = synth.workload(2, seed=1)
    print(f"generated {g.name} n={g.n} m={g.m} ({time.time() - t0:.0f} s)", flush=True)
    phase, center, order, P = oracle.schedule(g.n, g.src, g.dst, 16)
    print(f"schedule: {P} phases ({time.time() - t0:.0f} s)", flush=True)
    x, L = oracle.init(g.n, g.src, g.dst, g.w)
    T = 22
    oracle.sweep(g.n, g.src, g.dst, g.w, order, T, x, L)
    D, s, _ = oracle.stats(L)
    ex = oracle.extract(g.n, g.src, g.dst, g.w, L)
    print(f"{T} sweeps, D {D}, densest prefix {ex['num_w']}/{ex['den']} "
          f"({time.time() - t0:.0f} s)", flush=True)
    rng = np.random.default_rng(2307)
    top = np.argsort(-L, kind="stable")[:2048]
    rest = np.setdiff1d(np.arange(g.n), top)
    pick = np.sort(np.concatenate([top, rng.choice(rest, 2048, replace=False)]))
    out = {
        "source": "written by tests/golden/make_chunglu4m.py from synth and the oracle alone",
        "workload": g.name,
        "n": g.n,
        "m": g.m,
        "star_max": 16,
        "phases": P,
        "sweeps": T,
        "loads_sha256": digest(L),
        "fractions_sha256": digest(x),
        "D": float(D).hex(),
        "load_sum": float(s).hex(),
        "sample_nodes": [int(v) for v in pick],
        "sample_loads": [float(L[v]).hex() for v in pick],
        "extract": {"num": int(ex["num"]), "num_w": float(ex["num_w"]).hex(),
                    "den": int(ex["den"]),
                    "in_set_sha256": digest(ex["in_set"].astype(np.uint8))},
    }
    with open(os.path.join(HERE, "chunglu4m.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")
    print("wrote chunglu4m.json", flush=True)


if __name__ == "__main__":
    main()
