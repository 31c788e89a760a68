"""Python access to the plain FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library or its binding.  The
oracle shares no code with the GPU path; it follows the paper's Algorithm 1
(LOWD) and Algorithm 2 (Pruning) step by step, sequentially, in FP64.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")


def build(force: bool = True) -> str:
    """Compile oracle.c with gcc; -ffp-contract=off keeps every product and
    sum rounded on its own, exactly as written."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
                               "-Wall", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        lib = C.CDLL(_LIB)
        i64 = C.c_int64
        fptr = C.c_void_p
        lib.oracle_prune.argtypes = [i64, i64, _i32p, _i32p, _u8p, C.POINTER(C.c_int32),
                                     C.POINTER(i64), C.POINTER(i64)]
        lib.oracle_schedule.argtypes = [i64, i64, _i32p, _i32p, C.c_int32, _i32p, _i32p, _i32p,
                                        C.POINTER(C.c_int32)]
        lib.oracle_init.argtypes = [i64, i64, _i32p, _i32p, fptr, _f64p, _f64p]
        lib.oracle_sweep.argtypes = [i64, i64, _i32p, _i32p, fptr, _i32p, i64, C.c_int32, _f64p, _f64p]
        lib.oracle_stats.argtypes = [i64, _f64p, C.POINTER(C.c_double), C.POINTER(C.c_double),
                                     C.POINTER(C.c_double)]
        lib.oracle_extract.argtypes = [i64, i64, _i32p, _i32p, fptr, _f64p, _u8p, C.POINTER(i64),
                                       C.POINTER(i64), C.POINTER(C.c_double), C.POINTER(i64)]
        lib.oracle_ldd.argtypes = [i64, i64, _i32p, _i32p, fptr, _f64p, _i32p, _i64p, _f64p,
                                   C.POINTER(i64)]
        lib.oracle_greedy.argtypes = [i64, i64, _i32p, _i32p, _i32p, _i64p, C.POINTER(i64)]
        for f in (lib.oracle_prune, lib.oracle_schedule, lib.oracle_init, lib.oracle_sweep,
                  lib.oracle_stats, lib.oracle_extract, lib.oracle_ldd, lib.oracle_greedy):
            f.restype = C.c_int
        _lib = lib
    return _lib


def _wptr(w: Optional[np.ndarray]):
    if w is None:
        return None, None
    w = np.ascontiguousarray(w, dtype=np.float32)
    return w, w.ctypes.data_as(C.c_void_p)


def _check(rc: int, what: str):
    if rc != 0:
        raise RuntimeError(f"{what} failed with status {rc}")


def prune(n: int, src: np.ndarray, dst: np.ndarray):
    """Algorithm 2 on an unweighted graph -> (node_keep u8[n], rounds, n_h, m_h)."""
    lib = _load()
    keep = np.zeros(n, dtype=np.uint8)
    r = C.c_int32(0)
    nh = C.c_int64(0)
    mh = C.c_int64(0)
    _check(lib.oracle_prune(n, src.size, src, dst, keep, C.byref(r), C.byref(nh), C.byref(mh)),
           "oracle_prune")
    return keep, int(r.value), int(nh.value), int(mh.value)


def schedule(n: int, src: np.ndarray, dst: np.ndarray, smax: int = 16):
    """Phase schedule -> (phase i32[m], center i32[m], order i32[m], nphases)."""
    lib = _load()
    m = src.size
    phase = np.zeros(m, dtype=np.int32)
    center = np.zeros(m, dtype=np.int32)
    order = np.zeros(m, dtype=np.int32)
    P = C.c_int32(0)
    _check(lib.oracle_schedule(n, m, src, dst, smax, phase, center, order, C.byref(P)),
           "oracle_schedule")
    return phase, center, order, int(P.value)


def init(n: int, src: np.ndarray, dst: np.ndarray, w: Optional[np.ndarray]):
    """Algorithm 1 initialisation -> (x f64[m], L f64[n])."""
    lib = _load()
    m = src.size
    x = np.zeros(m, dtype=np.float64)
    L = np.zeros(n, dtype=np.float64)
    w, wp = _wptr(w)
    _check(lib.oracle_init(n, m, src, dst, wp, x, L), "oracle_init")
    return x, L


def sweep(n: int, src: np.ndarray, dst: np.ndarray, w: Optional[np.ndarray], order: np.ndarray,
          T: int, x: np.ndarray, L: np.ndarray) -> None:
    """T sweeps of the locally optimal step over `order`, in place on x, L."""
    lib = _load()
    w, wp = _wptr(w)
    order = np.ascontiguousarray(order, dtype=np.int32)
    _check(lib.oracle_sweep(n, src.size, src, dst, wp, order, order.size, T, x, L),
           "oracle_sweep")


def stats(L: np.ndarray):
    """(D = max load, sum of loads, sum of squared loads)."""
    lib = _load()
    D = C.c_double(0)
    s = C.c_double(0)
    s2 = C.c_double(0)
    _check(lib.oracle_stats(L.size, L, C.byref(D), C.byref(s), C.byref(s2)), "oracle_stats")
    return D.value, s.value, s2.value


def extract(n: int, src: np.ndarray, dst: np.ndarray, w: Optional[np.ndarray], L: np.ndarray):
    """Sort-and-peel extraction -> dict(in_set u8[n], best_i, num, num_w, den)."""
    lib = _load()
    in_set = np.zeros(n, dtype=np.uint8)
    bi = C.c_int64(0)
    nu = C.c_int64(0)
    nw = C.c_double(0)
    den = C.c_int64(0)
    w, wp = _wptr(w)
    _check(lib.oracle_extract(n, src.size, src, dst, wp, L, in_set, C.byref(bi), C.byref(nu),
                              C.byref(nw), C.byref(den)), "oracle_extract")
    return dict(in_set=in_set, best_i=int(bi.value), num=int(nu.value), num_w=float(nw.value),
                den=int(den.value))


def greedy(n: int, src: np.ndarray, dst: np.ndarray):
    """Greedy peeling (Algorithm 3) -> dict(order int32[n], rem_m int64[n],
    best_i, num, den, in_set uint8[n]): S* = V minus the first best_i
    removed nodes, with num = |E(S*)| and den = |S*|."""
    lib = _load()
    order = np.zeros(n, dtype=np.int32)
    rem_m = np.zeros(n, dtype=np.int64)
    bi = C.c_int64(0)
    _check(lib.oracle_greedy(n, src.size, np.ascontiguousarray(src, np.int32),
                             np.ascontiguousarray(dst, np.int32), order, rem_m, C.byref(bi)),
           "oracle_greedy")
    b = int(bi.value)
    in_set = np.ones(n, dtype=np.uint8)
    in_set[order[:b]] = 0
    num = int(src.size) if b == 0 else int(rem_m[b - 1])
    return dict(order=order, rem_m=rem_m, best_i=b, num=num, den=n - b, in_set=in_set)


def prune_weighted(n: int, src: np.ndarray, dst: np.ndarray, w: np.ndarray):
    """Algorithm 2 on a weighted graph, in exact rational arithmetic (plain
    Python; small graphs only).  H <- G; each round computes every node's
    weighted degree in H and the density rho(H) = w(E(H)) / |V(H)|, and
    removes every node with degree < rho(H) (decided exactly on the given
    float32 weights); it stops when a round removes nothing.  Isolated nodes
    count in |V(H)|.  Returns (node_keep uint8[n], rounds, n_h, m_h, w(E(H)))."""
    from fractions import Fraction
    wf = [Fraction(float(x)) for x in np.asarray(w, dtype=np.float32)]
    s = [int(a) for a in src]
    d = [int(b) for b in dst]
    alive = [True] * n
    rounds = 0
    while True:
        N = sum(alive)
        deg = [Fraction(0)] * n
        W = Fraction(0)
        for e in range(len(s)):
            if alive[s[e]] and alive[d[e]]:
                deg[s[e]] += wf[e]
                deg[d[e]] += wf[e]
                W += wf[e]
        gone = [u for u in range(n) if alive[u] and deg[u] * N < W]
        if not gone:
            break
        for u in gone:
            alive[u] = False
        rounds += 1
    keep = np.array(alive, dtype=np.uint8)
    m_h = sum(1 for e in range(len(s)) if alive[s[e]] and alive[d[e]])
    return keep, rounds, int(keep.sum()), m_h, W


def ldd(n: int, src: np.ndarray, dst: np.ndarray, w: Optional[np.ndarray], L: np.ndarray):
    """Locally-dense decomposition read from loads L (prefixes of the
    descending load order) -> dict(level int32[n], k_end int64[L], f_end
    float64[L]); lambda_j = (f_end[j] - f_end[j-1]) / (k_end[j] - k_end[j-1])."""
    lib = _load()
    level = np.zeros(n, dtype=np.int32)
    k_end = np.zeros(max(n, 1), dtype=np.int64)
    f_end = np.zeros(max(n, 1), dtype=np.float64)
    nl = C.c_int64(0)
    w, wp = _wptr(w)
    _check(lib.oracle_ldd(n, src.size, src, dst, wp, np.ascontiguousarray(L, dtype=np.float64),
                          level, k_end, f_end, C.byref(nl)), "oracle_ldd")
    k = int(nl.value)
    return dict(level=level, k_end=k_end[:k], f_end=f_end[:k])


def dks_bound(k_end: np.ndarray, f_end: np.ndarray, k: int) -> float:
    """Corollary 1: an upper bound on the density of any k-node subgraph from
    the decomposition's levels (the concave envelope of f at k, over k); at
    k = |B_j| it is the density of B_j itself."""
    kp, fp = 0, 0.0
    for kj, fj in zip(k_end, f_end):
        if k <= kj:
            return (fp + (k - kp) * (fj - fp) / (kj - kp)) / k
        kp, fp = int(kj), float(fj)
    raise ValueError("k exceeds the node count")


def solve(n: int, src: np.ndarray, dst: np.ndarray, w: Optional[np.ndarray], T: int,
          smax: int = 16):
    """Init, T sweeps in schedule order, extraction, statistics."""
    phase, center, order, P = schedule(n, src, dst, smax)
    x, L = init(n, src, dst, w)
    sweep(n, src, dst, w, order, T, x, L)
    ex = extract(n, src, dst, w, L)
    D, s, s2 = stats(L)
    rho = (ex["num"] if w is None else ex["num_w"]) / ex["den"]
    ex.update(x=x, L=L, D=D, sumL=s, sumL2=s2, rho=rho, gap=(D - rho) / rho, order=order,
              phase=phase, nphases=P)
    return ex
