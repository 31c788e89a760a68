"""Seeded synthetic graph generators shared by the tests, the benchmark and the
oracle's callers.

This module holds no part of the densest-subgraph method: it only draws graphs.
Every graph comes back in the canonical form the method assumes (Section IV,
experimental setup: multi-edges and self-loops removed, direction ignored):

    n    : number of nodes, ids in [0, n)
    src  : int32[m], dst : int32[m] with src < dst, sorted by (src, dst),
           no duplicate pair
    w    : None (unit weights) or float32[m] > 0

The workloads stand in for the paper's real datasets (Table I: social,
citation and rating graphs of 10^5 to 2.6*10^8 edges), which are not
available; their shapes (power-law degrees, a planted dense block, R-MAT
skew, many small graphs of uneven size) follow the configurations the
benchmark is quoted on.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import List, Optional

import numpy as np


@dataclass
class Graph:
    n: int
    src: np.ndarray            # int32[m]
    dst: np.ndarray            # int32[m]
    w: Optional[np.ndarray]    # float32[m] or None (unit weights)
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.src.shape[0])


def canonical(n: int, a: np.ndarray, b: np.ndarray, w: Optional[np.ndarray] = None,
              name: str = "") -> Graph:
    """Drop self-loops, ignore direction, drop repeated pairs (the first
    occurrence's weight is kept), sort by (min, max)."""
    a = np.asarray(a, dtype=np.int64)
    b = np.asarray(b, dtype=np.int64)
    keep = a != b
    a, b = a[keep], b[keep]
    if w is not None:
        w = np.asarray(w)[keep]
    lo = np.minimum(a, b)
    hi = np.maximum(a, b)
    key = lo * np.int64(n) + hi
    _, first = np.unique(key, return_index=True)   # sorted by key
    src = (key[first] // n).astype(np.int32)
    dst = (key[first] % n).astype(np.int32)
    ww = None
    if w is not None:
        ww = np.ascontiguousarray(np.asarray(w)[first], dtype=np.float32)
    return Graph(int(n), np.ascontiguousarray(src), np.ascontiguousarray(dst), ww, name)


def _distinct_pairs(rng: np.random.Generator, n: int, m: int) -> tuple:
    """m distinct unordered pairs of distinct nodes, uniformly at random."""
    out = np.empty(0, dtype=np.int64)
    total = n * (n - 1) // 2
    if m > total:
        raise ValueError("more edges than pairs")
    while out.size < m:
        need = (m - out.size) * 2 + 16
        a = rng.integers(0, n, size=need, dtype=np.int64)
        b = rng.integers(0, n, size=need, dtype=np.int64)
        ok = a != b
        lo = np.minimum(a[ok], b[ok])
        hi = np.maximum(a[ok], b[ok])
        key = np.concatenate([out, lo * n + hi])
        _, idx = np.unique(key, return_index=True)
        out = key[np.sort(idx)]     # keep draw order, drop repeats
    out = out[:m]
    return out // n, out % n


def erdos_renyi_planted(n: int = 1000, m: int = 5000, clique: int = 30, seed: int = 1) -> Graph:
    """G(n, m) on distinct uniform pairs plus a clique on `clique` random
    nodes (the small correctness workload: about 5.4k edges)."""
    rng = np.random.default_rng(seed)
    a, b = _distinct_pairs(rng, n, m)
    members = rng.choice(n, size=clique, replace=False)
    iu, ju = np.triu_indices(clique, 1)
    a = np.concatenate([a, members[iu]])
    b = np.concatenate([b, members[ju]])
    return canonical(n, a, b, None, f"er{n}_{m}+K{clique}")


def _chung_lu_weights(n: int, m: int, beta: float, cap: Optional[float]) -> np.ndarray:
    """Expected degrees proportional to (i+1)^(-1/(beta-1)), scaled to mean
    2m/n, then capped (the cap keeps expected degrees below sqrt(2m))."""
    i = np.arange(n, dtype=np.float64)
    raw = (i + 1.0) ** (-1.0 / (beta - 1.0))
    wts = raw * (2.0 * m / n) / raw.mean()
    if cap is not None:
        wts = np.minimum(wts, cap)
    return wts


def _sample_endpoints(rng: np.random.Generator, cdf: np.ndarray, k: int) -> np.ndarray:
    u = rng.random(k)
    return np.searchsorted(cdf, u, side="right").astype(np.int64)


def chung_lu(n: int, m: int, beta: float, seed: int, planted: int = 0, p_planted: float = 0.0,
             weights: str = "unit", cap: Optional[float] = -1.0, name: str = "") -> Graph:
    """Chung-Lu power-law graph: m endpoint pairs drawn with probability
    proportional to the expected-degree weights, self-loops and repeats
    dropped; optionally a planted block of `planted` random nodes whose pairs
    are present with probability p_planted; node ids randomly permuted.

    weights="lognormal" draws one lognormal(0, 1) weight per unique edge and
    rounds it to float32, so FP32 and FP64 consumers see identical values.
    cap=-1 means the default cap sqrt(2m); None means no cap."""
    rng = np.random.default_rng(seed)
    if cap is not None and cap < 0:
        cap = math.sqrt(2.0 * m)
    wts = _chung_lu_weights(n, m, beta, cap)
    cdf = np.cumsum(wts)
    cdf /= cdf[-1]
    a = np.empty(m, dtype=np.int64)
    b = np.empty(m, dtype=np.int64)
    chunk = 1 << 24
    for s in range(0, m, chunk):
        k = min(chunk, m - s)
        a[s:s + k] = _sample_endpoints(rng, cdf, k)
        b[s:s + k] = _sample_endpoints(rng, cdf, k)
    np.minimum(a, n - 1, out=a)
    np.minimum(b, n - 1, out=b)
    if planted > 0:
        members = rng.choice(n, size=planted, replace=False)
        iu, ju = np.triu_indices(planted, 1)
        pick = rng.random(iu.size) < p_planted
        a = np.concatenate([a, members[iu[pick]]])
        b = np.concatenate([b, members[ju[pick]]])
    perm = rng.permutation(n).astype(np.int64)
    a = perm[a]
    b = perm[b]
    g = canonical(n, a, b, None, name or f"chunglu{n}_{m}_b{beta}")
    if weights == "lognormal":
        g.w = rng.lognormal(0.0, 1.0, size=g.m).astype(np.float32)
        # guard: every weight strictly positive after rounding
        g.w[g.w <= 0] = np.float32(np.finfo(np.float32).tiny)
    elif weights != "unit":
        raise ValueError(weights)
    return g


_M64 = (1 << 64) - 1


def _s64(c: int) -> int:
    """A 64-bit constant as the signed value torch's int64 holds."""
    return c - (1 << 64) if c >= (1 << 63) else c


def _mix64(torch, z):
    """SplitMix64's output mix (Steele, Lea and Flood 2014) on an int64
    tensor, with logical right shifts; products wrap modulo 2^64 on every
    device, so CPU and GPU give the same bits."""
    z = z ^ ((z >> 30) & ((1 << 34) - 1))
    z = z * _s64(0xBF58476D1CE4E5B9)
    z = z ^ ((z >> 27) & ((1 << 37) - 1))
    z = z * _s64(0x94D049BB133111EB)
    return z ^ ((z >> 31) & ((1 << 33) - 1))


def _hash_stream(torch, seed: int, stream: int, index):
    """Counter-based random words: the SplitMix64 mix of (seed, stream,
    index), so any element can be drawn on its own, on any device."""
    return _mix64(torch, index * _s64(0x9E3779B97F4A7C15) + _s64(_mix64_int(seed, stream)))


def _mix64_int(seed: int, stream: int) -> int:
    """The stream's offset: SplitMix64's mix of (seed, stream) in Python
    integers, so that streams are unrelated (not shifted copies)."""
    z = (((seed & 0xFFFFFFFF) << 32) | (stream & 0xFFFFFFFF)) * 0x9E3779B97F4A7C15 & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def rmat(scale: int, edge_factor: int = 16, a: float = 0.57, b: float = 0.19, c: float = 0.19,
         seed: int = 1, permute: bool = True, samples: Optional[int] = None,
         device: str = "cpu") -> Graph:
    """R-MAT: `edge_factor * 2^scale` samples; at each of the `scale` levels
    a sample picks quadrant (0,0), (0,1), (1,0), (1,1) with probabilities
    (a, b, c, d = 1-a-b-c), each level from 16 random bits (probabilities
    rounded to multiples of 2^-16), no noise; node ids permuted by a random
    permutation; symmetrised and de-duplicated.  The random bits are a
    counter-based hash, so the graph is the same on the CPU and on a GPU
    (device="cuda" draws 2^28 samples in about a second)."""
    import torch
    n = 1 << scale
    k_total = samples if samples is not None else edge_factor * n
    ta = int(round(a * 65536))
    tab = int(round((a + b) * 65536))
    tabc = int(round((a + b + c) * 65536))
    words = (scale + 3) // 4            # 64 bits = four 16-bit draws per word
    keys = []
    chunk = 1 << 26
    for s0 in range(0, k_total, chunk):
        k = min(chunk, k_total - s0)
        idx = torch.arange(s0, s0 + k, dtype=torch.int64, device=device)
        u = torch.zeros(k, dtype=torch.int64, device=device)
        v = torch.zeros(k, dtype=torch.int64, device=device)
        lvl = 0
        for j in range(words):
            h = _hash_stream(torch, seed, 1 + j, idx)
            for q in range(4):
                if lvl == scale:
                    break
                r = (h >> (16 * q)) & 0xFFFF
                ubit = (r >= tab).to(torch.int64)
                vbit = (((r >= ta) & (r < tab)) | (r >= tabc)).to(torch.int64)
                u = (u << 1) | ubit
                v = (v << 1) | vbit
                lvl += 1
        keep = u != v
        u, v = u[keep], v[keep]
        if permute:
            if s0 == 0:
                nodes = torch.arange(n, dtype=torch.int64, device=device)
                perm = torch.argsort(_hash_stream(torch, seed, 0, nodes), stable=True)
            u = perm[u]
            v = perm[v]
        lo = torch.minimum(u, v)
        hi = torch.maximum(u, v)
        keys.append(torch.unique(lo * n + hi))
        del idx, u, v, lo, hi
    key = torch.unique(torch.cat(keys)) if len(keys) > 1 else keys[0]
    del keys
    src = (key // n).to(torch.int32).cpu().numpy()
    dst = (key % n).to(torch.int32).cpu().numpy()
    return Graph(int(n), np.ascontiguousarray(src), np.ascontiguousarray(dst), None,
                 f"rmat{scale}_{edge_factor}")


def batch_of_graphs(count: int = 4096, seed: int = 1, m_lo: int = 100, m_hi: int = 50000,
                    beta: float = 2.3) -> List[Graph]:
    """Many independent uneven graphs: edge targets log-uniform in
    [m_lo, m_hi]; n = max(s + 8, m/4); Chung-Lu exponent beta background plus
    a planted block of s ~ U{5..40} nodes with pair probability 0.5 (s capped
    so the planted pairs stay below half the edge target)."""
    rng = np.random.default_rng(seed)
    out = []
    for gi in range(count):
        mt = int(round(math.exp(rng.uniform(math.log(m_lo), math.log(m_hi)))))
        s = int(rng.integers(5, 41))
        while s > 2 and 0.5 * s * (s - 1) / 2 > mt / 2:
            s -= 1
        n = max(s + 8, int(round(mt / 4)))
        members = rng.choice(n, size=s, replace=False)
        iu, ju = np.triu_indices(s, 1)
        pick = rng.random(iu.size) < 0.5
        pa, pb = members[iu[pick]], members[ju[pick]]
        bg = max(mt - int(pick.sum()), 1)
        wts = _chung_lu_weights(n, bg, beta, math.sqrt(2.0 * bg))
        cdf = np.cumsum(wts)
        cdf /= cdf[-1]
        a = np.minimum(_sample_endpoints(rng, cdf, bg), n - 1)
        b = np.minimum(_sample_endpoints(rng, cdf, bg), n - 1)
        perm = rng.permutation(n).astype(np.int64)
        a = np.concatenate([perm[a], pa])
        b = np.concatenate([perm[b], pb])
        out.append(canonical(n, a, b, None, f"batch{gi}"))
    return out


def uniform_pairs(log_n: int = 22, log_m: int = 28, seed: int = 1, device: str = "cpu") -> Graph:
    """2^log_m uniform random pairs on 2^log_n nodes, self-loops and repeats
    dropped: a graph of small maximum degree, whose sweep phases are few and
    wide (a diagnostic of the sweep's memory bandwidth, not one of the paper's
    workloads).  Counter-based random bits, as for rmat()."""
    import torch
    n, m = 1 << log_n, 1 << log_m
    keys = []
    chunk = 1 << 26
    for s0 in range(0, m, chunk):
        k = min(chunk, m - s0)
        idx = torch.arange(s0, s0 + k, dtype=torch.int64, device=device)
        h = _hash_stream(torch, seed, 100, idx)
        a = h & (n - 1)
        b = (h >> 32) & (n - 1)
        keep = a != b
        a, b = a[keep], b[keep]
        keys.append(torch.unique(torch.minimum(a, b) * n + torch.maximum(a, b)))
    key = torch.unique(torch.cat(keys)) if len(keys) > 1 else keys[0]
    src = (key // n).to(torch.int32).cpu().numpy()
    dst = (key % n).to(torch.int32).cpu().numpy()
    return Graph(int(n), np.ascontiguousarray(src), np.ascontiguousarray(dst), None,
                 f"uniform_2^{log_n}_2^{log_m}")


def random_small(rng: np.random.Generator, n: int, p: float, weighted: bool = False) -> Graph:
    """G(n, p) for brute-force checks; optional weights in {1..4}/2 (exact in
    binary floating point) or lognormal."""
    iu, ju = np.triu_indices(n, 1)
    pick = rng.random(iu.size) < p
    a, b = iu[pick], ju[pick]
    w = None
    if weighted:
        w = rng.integers(1, 5, size=a.size).astype(np.float32) / np.float32(2.0)
    return canonical(n, a, b, w, f"gnp{n}_{p}")


# The workloads, by their sizes.  Index 0 is the small correctness case.
def workload(k: int, seed: int = 1):
    if k == 0:
        return erdos_renyi_planted(1000, 5000, 30, seed)
    if k == 1:
        return chung_lu(1_000_000, 10_000_000, 2.1, seed, planted=500, p_planted=0.3,
                        name="chunglu_1M_10M_b2.1")
    if k == 2:
        return chung_lu(4_000_000, 64_000_000, 2.1, seed, planted=500, p_planted=0.3,
                        weights="lognormal", name="chunglu_4M_64M_b2.1_lognormal")
    if k == 3:
        return rmat(24, 16, seed=seed)
    if k == 4:
        return batch_of_graphs(4096, seed)
    raise ValueError(k)
