"""Writes rmat24_h.json: the oracle's results on the R-MAT scale 24 workload,
for the full-size GPU test (tests/test_gpu_parity.py,
test_rmat24_full_size_prune_and_three_sweeps).

Only the seeded input generator (synth) and the oracle run here:
  1. R-MAT scale 24, edge factor 16, seed 1 (16.8M nodes, 260M edges);
  2. oracle.prune (Algorithm 2): rounds, |V(H)|, |E(H)| and a digest of
     the node mask;
  3. H's edge list in H's ids, the kept edges in their original order;
  4. oracle.schedule with stars of at most 32 leaves, oracle.init, three
     oracle sweeps (Algorithm 1), digests of the loads and fractions, and
     oracle.extract on those loads (the densest prefix, exact rational).
The oracle's schedule is its plain sequential first fit: about 4 minutes
on R-MAT 24's H.  Run from the repository root:
    python tests/golden/make_rmat24_h.py
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
    g = synth.rmat(24, 16, seed=1)
    print(f"generated n={g.n} m={g.m} ({time.time() - t0:.0f} s)", flush=True)
    keep, rounds, nh, mh = oracle.prune(g.n, g.src, g.dst)
    print(f"pruned: rounds {rounds}, H {nh} / {mh} ({time.time() - t0:.0f} s)", flush=True)
    kept = (keep[g.src] == 1) & (keep[g.dst] == 1)
    newid = np.cumsum(keep.astype(np.int64)) - 1
    hs = np.ascontiguousarray(newid[g.src[kept]].astype(np.int32))
    hd = np.ascontiguousarray(newid[g.dst[kept]].astype(np.int32))
    del g, kept, newid
    phase, center, order, P = oracle.schedule(nh, hs, hd, 32)
    print(f"schedule: {P} phases ({time.time() - t0:.0f} s)", flush=True)
    x, L = oracle.init(nh, hs, hd, None)
    T = 3
    oracle.sweep(nh, hs, hd, None, order, T, x, L)
    ex = oracle.extract(nh, hs, hd, None, L)
    print(f"{T} sweeps, densest prefix {ex['num']}/{ex['den']} ({time.time() - t0:.0f} s)",
          flush=True)
    out = {
        "source": "written by tests/golden/make_rmat24_h.py from synth and the oracle alone",
        "workload": "R-MAT scale 24, edge factor 16, (a, b, c) = (0.57, 0.19, 0.19), seed 1",
        "n": 1 << 24,
        "prune": {"rounds": rounds, "n_h": nh, "m_h": mh, "node_keep_sha256": digest(keep)},
        "star_max": 32,
        "phases": P,
        "sweeps": T,
        "loads_sha256": digest(L),
        "fractions_sha256": digest(x),
        "extract": {"num": int(ex["num"]), "den": int(ex["den"]),
                    "in_set_sha256": digest(ex["in_set"].astype(np.uint8))},
    }
    with open(os.path.join(HERE, "rmat24_h.json"), "w") as f:
        json.dump(out, f, indent=2)
        f.write("\n")
    print("wrote rmat24_h.json", flush=True)


if __name__ == "__main__":
    main()
