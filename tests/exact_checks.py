"""Independent exact checkers used to pin the oracle.

None of this calls the oracle or the GPU library: these are textbook
definitions (brute force over subsets, Goldberg's max-flow construction,
greedy peeling, the k-core from networkx) evaluated with exact rationals or
integers where the inputs allow.
"""
from __future__ import annotations

import itertools
import math
from fractions import Fraction
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np


def _edges(src, dst, w):
    if w is None:
        return [(int(a), int(b), Fraction(1)) for a, b in zip(src, dst)]
    return [(int(a), int(b), Fraction(float(x))) for a, b, x in zip(src, dst, w)]


def induced_weight(edges, S: frozenset) -> Fraction:
    return sum((x for a, b, x in edges if a in S and b in S), Fraction(0))


def brute_force_densest(n: int, src, dst, w=None) -> Tuple[Fraction, frozenset]:
    """Maximum density over all non-empty subsets and the largest subset that
    reaches it (Problem 1; the union of two densest sets is densest)."""
    edges = _edges(src, dst, w)
    best = Fraction(-1)
    best_set = frozenset()
    for mask in range(1, 1 << n):
        S = frozenset(i for i in range(n) if mask >> i & 1)
        rho = induced_weight(edges, S) / len(S)
        if rho > best or (rho == best and len(S) > len(best_set)):
            best, best_set = rho, S
    return best, best_set


def brute_force_ldd(n: int, src, dst, w=None) -> Tuple[List[frozenset], List[Fraction]]:
    """Locally-dense decomposition by its definition (Section II): B_i is the
    maximal S properly containing B_{i-1} that maximises
    (W(S) - W(B_{i-1})) / |S minus B_{i-1}|.  Returns the nested sets and the
    per-node value lambda_u of the level u first enters."""
    edges = _edges(src, dst, w)
    prev = frozenset()
    levels = []
    lam = [Fraction(0)] * n
    full = frozenset(range(n))
    while prev != full:
        rest = sorted(full - prev)
        wprev = induced_weight(edges, prev)
        best = None
        best_set = None
        for mask in range(1, 1 << len(rest)):
            add = frozenset(rest[i] for i in range(len(rest)) if mask >> i & 1)
            S = prev | add
            val = (induced_weight(edges, S) - wprev) / len(add)
            if best is None or val > best or (val == best and len(S) > len(best_set)):
                best, best_set = val, S
        for u in best_set - prev:
            lam[u] = best
        levels.append(best_set)
        prev = best_set
    return levels, lam


def peel_densities(n: int, src, dst, w, order: Sequence[int]) -> List[Fraction]:
    """rho(S_i) for S_i = V minus the first i nodes of `order`, i = 0..n-1,
    by direct evaluation of every set."""
    edges = _edges(src, dst, w)
    out = []
    removed = set()
    for i in range(n):
        S = frozenset(set(range(n)) - removed)
        out.append(induced_weight(edges, S) / len(S))
        removed.add(order[i])
    return out


def goldberg_check(n: int, src, dst, num: int, den: int):
    """Goldberg's max-flow test for an unweighted graph at g = num/den.

    Network: source -> edge-node (capacity den), edge-node -> both endpoints
    (infinite), node -> sink (capacity num).  A minimum cut's source side is
    a set S with its induced edges, and
        max_S (den*|E(S)| - num*|S|) = den*m - maxflow.
    Returns (surplus, maximal_set): surplus == 0 means no set is denser than
    g; maximal_set is the largest S of zero surplus (the nodes that cannot
    reach the sink in the residual network)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import maximum_flow, breadth_first_order

    src = np.asarray(src, dtype=np.int64)
    dst = np.asarray(dst, dtype=np.int64)
    m = src.size
    g = math.gcd(num, den)
    p, q = num // g, den // g
    S, T = 0, m + n + 1
    big = q * m + 1
    e_nodes = np.arange(1, m + 1, dtype=np.int64)
    rows = np.concatenate([np.zeros(m, np.int64), e_nodes, e_nodes, 1 + m + np.arange(n)])
    cols = np.concatenate([e_nodes, 1 + m + src, 1 + m + dst, np.full(n, T)])
    caps = np.concatenate([np.full(m, q), np.full(2 * m, big), np.full(n, p)]).astype(np.int64)
    if caps.max() >= 2 ** 31:
        raise ValueError("capacities exceed int32")
    N = m + n + 2
    C = csr_matrix((caps.astype(np.int32), (rows, cols)), shape=(N, N))
    res = maximum_flow(C, S, T, method="dinic")
    surplus = q * m - int(res.flow_value)
    F = res.flow.tocsr()
    # residual capacities: C - F (F is antisymmetric, so reverse arcs appear)
    R = (C.astype(np.int64) - F.astype(np.int64)).tocsr()
    R.data[R.data < 0] = 0
    R.eliminate_zeros()
    # nodes that can reach the sink: BFS from T on the reversed residual graph
    reach = breadth_first_order(R.T.tocsr(), T, directed=True, return_predecessors=False)
    can_reach = np.zeros(N, dtype=bool)
    can_reach[reach] = True
    maximal = frozenset(int(u) for u in range(n) if not can_reach[1 + m + u])
    return surplus, maximal


def greedy_peel(n: int, src, dst) -> Tuple[List[Tuple[int, int]], List[int]]:
    """Charikar's greedy peeling (Appendix, Algorithm 3) on an unweighted
    graph: repeatedly remove a node of minimum degree (smallest id on ties).
    Returns the (|E|, |V|) of every remaining graph, starting with G, and the
    removal order."""
    adj = [set() for _ in range(n)]
    for a, b in zip(src, dst):
        adj[int(a)].add(int(b))
        adj[int(b)].add(int(a))
    alive = set(range(n))
    M = len(src)
    sizes = [(M, n)]
    order = []
    import heapq
    heap = [(len(adj[u]), u) for u in range(n)]
    heapq.heapify(heap)
    deg = [len(adj[u]) for u in range(n)]
    while alive:
        d, u = heapq.heappop(heap)
        if u not in alive or d != deg[u]:
            continue
        alive.remove(u)
        order.append(u)
        M -= deg[u]
        for v in adj[u]:
            if v in alive:
                deg[v] -= 1
                heapq.heappush(heap, (deg[v], v))
        if alive:
            sizes.append((M, len(alive)))
    return sizes, order


def greedy_peel_weighted(n: int, src, dst, w) -> Tuple[List[Tuple[Fraction, int]], List[int]]:
    """Greedy peeling on a weighted graph in exact arithmetic: repeatedly
    remove a node of minimum weighted degree (smallest id on ties).  Returns
    (w(E), |V|) of every remaining graph, starting with G, and the order."""
    wf = [Fraction(float(x)) for x in np.asarray(w, dtype=np.float32)]
    adj = [dict() for _ in range(n)]
    for e, (a, b) in enumerate(zip(src, dst)):
        adj[int(a)][int(b)] = wf[e]
        adj[int(b)][int(a)] = wf[e]
    deg = [sum(adj[u].values(), Fraction(0)) for u in range(n)]
    alive = set(range(n))
    W = sum(wf, Fraction(0))
    sizes = [(W, n)]
    order = []
    while alive:
        u = min(alive, key=lambda v: (deg[v], v))
        alive.remove(u)
        order.append(u)
        W -= deg[u]
        for v, x in adj[u].items():
            if v in alive:
                deg[v] -= x
        if alive:
            sizes.append((W, len(alive)))
    return sizes, order
