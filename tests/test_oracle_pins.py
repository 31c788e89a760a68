"""Pins of the FP64 CPU oracle against values the paper and the mathematics
fix, independently of the oracle's own code: the paper's worked step
(Fig. 1), closed forms, brute force over subsets, Goldberg's max-flow,
networkx's k-core, greedy peeling, and the invariants the paper proves
(Section III)."""
import json
import math
import os
from fractions import Fraction

import networkx as nx
import numpy as np
import pytest

import oracle
import synth
from exact_checks import (brute_force_densest, brute_force_ldd, goldberg_check, greedy_peel,
                          greedy_peel_weighted, peel_densities)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def graph_from_edges(n, edges, w=None):
    a = np.array([e[0] for e in edges], dtype=np.int64)
    b = np.array([e[1] for e in edges], dtype=np.int64)
    return synth.canonical(n, a, b, None if w is None else np.asarray(w, np.float32))


def converge(g, T, smax=16):
    return oracle.solve(g.n, g.src, g.dst, g.w, T, smax)


# ---------------------------------------------------------------- Fig. 1 --
def test_fig1_worked_step():
    """Section I, Fig. 1 (b)->(c): loads 2 and 1 both become 1.5; the edge
    goes entirely to node 6."""
    fx = json.load(open(os.path.join(GOLDEN, "fig1_step.json")))
    n = fx["n"]
    src = np.array([e[0] for e in fx["edges"]], dtype=np.int32)
    dst = np.array([e[1] for e in fx["edges"]], dtype=np.int32)
    x, L = oracle.init(n, src, dst, None)
    assert L[4] == fx["loads_before"]["4"] and L[6] == fx["loads_before"]["6"]
    oracle.sweep(n, src, dst, None, np.array([fx["step_edge"]], np.int32), 1, x, L)
    assert L[4] == fx["loads_after"]["4"] and L[6] == fx["loads_after"]["6"]
    e = fx["step_edge"]
    f4 = x[e] if src[e] == 4 else 1.0 - x[e]
    assert f4 == fx["fraction_after"]["f_e(4)"]
    # the other loads are untouched
    assert L[0] == 0.5 and L[3] == 0.5


# ------------------------------------------------------------ closed forms --
def test_init_unit_weights_is_half_degree():
    g = synth.workload(0)
    x, L = oracle.init(g.n, g.src, g.dst, None)
    deg = np.bincount(g.src, minlength=g.n) + np.bincount(g.dst, minlength=g.n)
    assert np.array_equal(L, deg / 2.0)
    assert np.all(x == 0.5)


@pytest.mark.parametrize("kind", ["cycle", "clique", "petersen", "hypercube"])
def test_regular_graph_is_a_fixed_point(kind):
    """All loads equal deg/2 at initialisation, so every step has d = 0 and
    the whole graph is densest with density deg/2."""
    G = {"cycle": nx.cycle_graph(11), "clique": nx.complete_graph(9),
         "petersen": nx.petersen_graph(), "hypercube": nx.hypercube_graph(4)}[kind]
    G = nx.convert_node_labels_to_integers(G)
    g = graph_from_edges(G.number_of_nodes(), list(G.edges()))
    r = converge(g, 5)
    k = 2 * g.m // g.n
    assert np.all(r["L"] == k / 2.0)
    assert np.all(r["x"] == 0.5)
    assert r["den"] == g.n and Fraction(r["num"], r["den"]) == Fraction(k, 2)


@pytest.mark.parametrize("k", [1, 2, 5, 12])
def test_star_limit(k):
    """K_{1,k}: the whole star is densest (density k/(k+1)), so every load
    tends to k/(k+1) (Property 2)."""
    g = graph_from_edges(k + 1, [(0, i) for i in range(1, k + 1)])
    r = converge(g, 4000)
    assert np.allclose(r["L"], k / (k + 1.0), rtol=0, atol=1e-9)
    assert r["den"] == k + 1


@pytest.mark.parametrize("nodes", [2, 3, 6, 9])
def test_path_limit(nodes):
    """Path P_n: a tree is densest as a whole, density (n-1)/n."""
    g = graph_from_edges(nodes, [(i, i + 1) for i in range(nodes - 1)])
    r = converge(g, 20000)
    assert np.allclose(r["L"], (nodes - 1) / nodes, rtol=0, atol=1e-9)


def test_two_equal_cliques_extract_both():
    """Two disjoint K_5 and a pendant path: the densest sets are either clique
    or both; the largest is returned (S* starts as V, replaced on a strict
    increase only)."""
    edges = [(a, b) for a in range(5) for b in range(a + 1, 5)]
    edges += [(a + 5, b + 5) for a in range(5) for b in range(a + 1, 5)]
    edges += [(10, 11), (11, 12), (12, 0)]
    g = graph_from_edges(13, edges)
    r = converge(g, 3000)
    assert set(np.flatnonzero(r["in_set"])) == set(range(10))
    assert Fraction(r["num"], r["den"]) == Fraction(2)


def test_barbell_is_uniform():
    """Two K_4 joined by one edge: density 13/8 exceeds each K_4's 6/4, so the
    whole graph is densest and every load tends to 13/8."""
    edges = [(a, b) for a in range(4) for b in range(a + 1, 4)]
    edges += [(a + 4, b + 4) for a in range(4) for b in range(a + 1, 4)]
    edges += [(3, 4)]
    g = graph_from_edges(8, edges)
    r = converge(g, 3000)
    assert np.allclose(r["L"], 13 / 8, atol=1e-12)
    assert r["den"] == 8


# ----------------------------------------------------- brute force, LDD --
def _random_graphs(count, nmin, nmax, weighted, seed):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        n = int(rng.integers(nmin, nmax + 1))
        g = synth.random_small(rng, n, float(rng.uniform(0.2, 0.7)), weighted)
        if g.m > 0:
            out.append(g)
    return out


@pytest.mark.parametrize("weighted", [False, True])
def test_limit_equals_brute_force_ldd(weighted):
    """Theorem 3 and Property 2: the converged loads equal the per-node value
    lambda of the locally-dense decomposition, computed from its definition."""
    for g in _random_graphs(25, 4, 9, weighted, 7 + weighted):
        _, lam = brute_force_ldd(g.n, g.src, g.dst, g.w)
        r = converge(g, 6000)
        lam = np.array([float(v) for v in lam])
        assert np.allclose(r["L"], lam, rtol=0, atol=1e-7), (g.src, g.dst, g.w, r["L"], lam)


@pytest.mark.parametrize("weighted", [False, True])
def test_extracted_set_is_maximal_densest_by_brute_force(weighted):
    """Problem 1: after convergence the extracted set is the largest densest
    set (B_1 of the decomposition)."""
    for g in _random_graphs(30, 3, 12, weighted, 11 + weighted):
        rho, S = brute_force_densest(g.n, g.src, g.dst, g.w)
        r = converge(g, 6000)
        got = frozenset(int(u) for u in np.flatnonzero(r["in_set"]))
        assert got == S, (g.src, g.dst, g.w)
        num = Fraction(r["num"]) if g.w is None else Fraction(r["num_w"])
        assert num / r["den"] == rho


def test_weighted_peel_densities_match_exact_evaluation():
    """Weighted graphs (float32 lognormal weights, no dyadic niceness): the
    oracle's choice of prefix is the first maximum of the exact rational
    densities (Problem 1), and its W is that exact rational rounded once."""
    rng = np.random.default_rng(17)
    for _ in range(20):
        n = int(rng.integers(3, 12))
        g = synth.random_small(rng, n, float(rng.uniform(0.3, 0.8)), False)
        if g.m == 0:
            continue
        w = rng.lognormal(0.0, 1.0, size=g.m).astype(np.float32)
        L = rng.integers(0, 3, size=g.n).astype(np.float64)       # many ties
        r = oracle.extract(g.n, g.src, g.dst, w, L)
        order = sorted(range(g.n), key=lambda u: (L[u], u))
        dens = peel_densities(g.n, g.src, g.dst, w, order)
        best = max(range(g.n), key=lambda i: (dens[i], -i))
        assert r["best_i"] == best
        assert r["num_w"] == float(dens[best] * (g.n - best))
        assert r["den"] == g.n - best


def test_weighted_exact_tie_keeps_the_larger_set():
    """Two disjoint triangles carry the same three float32 weights in
    different edge orders, so each has density 2 exactly and so does their
    union; among equally dense prefixes the largest is kept (S* is replaced
    only on a strict increase, O9), with the weights compared exactly."""
    src = np.array([0, 0, 1, 3, 3, 4, 6], dtype=np.int32)
    dst = np.array([1, 2, 2, 4, 5, 5, 7], dtype=np.int32)
    w = np.array([1.5, 2.0, 2.5, 2.5, 1.5, 2.0, 0.01], dtype=np.float32)
    n = 8
    L = np.array([1.0, 1.0, 1.0, 1.0, 1.0, 1.0, 0.0, 0.0])   # nodes 6, 7 go first
    r = oracle.extract(n, src, dst, w, L)
    assert list(np.flatnonzero(r["in_set"])) == [0, 1, 2, 3, 4, 5]
    assert r["num_w"] == 12.0 and r["den"] == 6
    # the prefix {3, 4, 5} ties with it and is not taken
    order = sorted(range(n), key=lambda u: (L[u], u))
    dens = peel_densities(n, src, dst, w, order)
    assert dens[2] == dens[5] == 2


def test_peel_densities_match_direct_evaluation():
    """The suffix-sum computation of rho(S_i) equals evaluating every S_i
    directly, for arbitrary (not converged) loads, including ties."""
    rng = np.random.default_rng(3)
    for g in _random_graphs(20, 3, 11, False, 5):
        L = rng.integers(0, 4, size=g.n).astype(np.float64) / 2.0   # many ties
        r = oracle.extract(g.n, g.src, g.dst, None, L)
        order = sorted(range(g.n), key=lambda u: (L[u], u))
        dens = peel_densities(g.n, g.src, g.dst, None, order)
        best = max(range(g.n), key=lambda i: (dens[i], -i))
        assert r["best_i"] == best
        assert Fraction(r["num"], r["den"]) == dens[best]
        assert set(np.flatnonzero(r["in_set"])) == set(order[best:])


# --------------------------------------------------------------- max-flow --
def test_config1_density_is_exact_by_maxflow():
    """ER(1000, 5000) plus a planted K_30, 200 sweeps (the small workload):
    the extracted density is rho* and the set is the maximal densest set,
    both certified by Goldberg's max-flow construction."""
    g = synth.workload(0)
    r = converge(g, 200)
    surplus, maximal = goldberg_check(g.n, g.src, g.dst, r["num"], r["den"])
    assert surplus == 0                       # no denser set exists
    assert frozenset(np.flatnonzero(r["in_set"]).tolist()) == maximal
    # the weak-duality sandwich rho_t <= rho* <= D_t, up to FP64 rounding of D
    assert r["rho"] <= r["D"] * (1 + 1e-12)


def test_maxflow_checker_agrees_with_brute_force():
    """The max-flow checker itself, on graphs small enough to enumerate."""
    for g in _random_graphs(15, 4, 11, False, 21):
        rho, S = brute_force_densest(g.n, g.src, g.dst)
        surplus, maximal = goldberg_check(g.n, g.src, g.dst, rho.numerator, rho.denominator)
        assert surplus == 0 and maximal == S
        # a slightly smaller guess leaves a positive surplus
        surplus2, _ = goldberg_check(g.n, g.src, g.dst, rho.numerator * 1000 - 1,
                                     rho.denominator * 1000)
        assert surplus2 > 0


# ---------------------------------------------------------------- pruning --
def _rho_h(keep, src, dst):
    inside = keep[src].astype(bool) & keep[dst].astype(bool)
    return Fraction(int(inside.sum()), max(int(keep.sum()), 1)), inside


@pytest.mark.parametrize("seed", range(6))
def test_prune_equals_core_of_ceil_density(seed):
    """Every removed node had degree below delta <= rho(H), every kept node
    has degree >= rho(H) (Theorem 4), so H is the ceil(rho(H))-core of G."""
    rng = np.random.default_rng(seed)
    for _ in range(20):
        n = int(rng.integers(5, 120))
        g = synth.random_small(rng, n, float(rng.uniform(0.02, 0.4)))
        if g.m == 0:
            continue
        keep, rounds, nh, mh = oracle.prune(g.n, g.src, g.dst)
        rho, inside = _rho_h(keep, g.src, g.dst)
        assert nh == int(keep.sum()) and mh == int(inside.sum())
        G = nx.Graph()
        G.add_nodes_from(range(g.n))
        G.add_edges_from(zip(g.src.tolist(), g.dst.tolist()))
        k = math.ceil(rho)
        core = set(nx.k_core(G, k).nodes())
        assert set(np.flatnonzero(keep)) == core


def test_prune_workload0_and_densest_inside():
    g = synth.workload(0)
    keep, rounds, nh, mh = oracle.prune(g.n, g.src, g.dst)
    G = nx.Graph()
    G.add_edges_from(zip(g.src.tolist(), g.dst.tolist()))
    rho, inside = _rho_h(keep, g.src, g.dst)
    assert set(np.flatnonzero(keep)) == set(nx.k_core(G, math.ceil(rho)).nodes())
    # Theorem 4 / Section III-D: the densest set survives pruning
    r = converge(g, 200)
    assert np.all(keep[r["in_set"].astype(bool)] == 1)
    # density of H is at least that of G
    assert rho >= Fraction(g.m, g.n)
    # minimum degree in H is at least rho(H)
    deg = np.bincount(g.src[inside], minlength=g.n) + np.bincount(g.dst[inside], minlength=g.n)
    assert deg[keep.astype(bool)].min() >= rho


def test_prune_matches_greedy_first_density_decrease():
    """Theorem 5 and Lemma 3: greedy peeling passes through the pruned graph H
    (the moment it first removes a node of H, exactly H remains), its density
    never decreases before that, and the first strict decrease comes at H or
    later.  (When greedy removes a node of degree exactly rho(H) the density
    stays equal, so "the first decrease" can come after H; the theorem's
    proof shows the monotone phase ends no earlier than H.)"""
    rng = np.random.default_rng(99)
    checked = 0
    for _ in range(60):
        n = int(rng.integers(8, 80))
        g = synth.random_small(rng, n, float(rng.uniform(0.05, 0.3)))
        if g.m == 0:
            continue
        keep, _, nh, mh = oracle.prune(g.n, g.src, g.dst)
        sizes, order = greedy_peel(g.n, g.src, g.dst)
        k = g.n - nh                       # removals before H is reached
        assert sizes[k] == (mh, nh)
        assert set(order[k:]) == set(np.flatnonzero(keep))
        dens = [Fraction(M, N) for M, N in sizes]
        assert all(dens[i + 1] >= dens[i] for i in range(k))
        first_dec = next((i for i in range(len(dens) - 1) if dens[i + 1] < dens[i]), len(dens))
        assert first_dec >= k
        checked += 1
    assert checked > 40


def test_prune_no_edges_keeps_everything():
    keep, rounds, nh, mh = oracle.prune(5, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert keep.tolist() == [1] * 5 and rounds == 0 and nh == 5 and mh == 0


# ------------------------------------------------------------- invariants --
def test_invariants_along_the_iteration():
    """Section III: f_e(u)+f_e(v) = w_e, 0 <= f <= w, sum of loads = sum of
    weights; D_t non-increasing (Theorem 1's monotonicity) and the QP
    objective sum l^2 non-increasing (Section III-C)."""
    rng = np.random.default_rng(4)
    for weighted in (False, True):
        g = synth.random_small(rng, 150, 0.08, weighted)
        wv = np.ones(g.m) if g.w is None else g.w.astype(np.float64)
        _, _, order, _ = oracle.schedule(g.n, g.src, g.dst, 16)
        x, L = oracle.init(g.n, g.src, g.dst, g.w)
        prevD, _, prevQ = oracle.stats(L)
        for t in range(60):
            oracle.sweep(g.n, g.src, g.dst, g.w, order, 1, x, L)
            D, s, Q = oracle.stats(L)
            assert np.all(x >= 0) and np.all(x <= wv)
            assert abs(s - wv.sum()) <= 1e-12 * wv.sum() * 10
            # monotone up to the rounding of a sum over n terms
            assert D <= prevD * (1 + 1e-13)
            assert Q <= prevQ * (1 + 1e-12)
            prevD, prevQ = D, Q
            # loads equal the sums of the fractions (up to rounding)
            Lr = np.zeros(g.n)
            np.add.at(Lr, g.src, x)
            np.add.at(Lr, g.dst, wv - x)
            assert np.allclose(Lr, L, rtol=0, atol=1e-10)


def test_each_step_never_increases_the_qp_objective():
    """One locally optimal step changes sum l^2 by 2d(d + l_v - l_u) <= 0."""
    rng = np.random.default_rng(8)
    g = synth.random_small(rng, 40, 0.2, True)
    x, L = oracle.init(g.n, g.src, g.dst, g.w)
    for i in range(400):
        e = int(rng.integers(0, g.m))
        q0 = float(np.dot(L, L))
        oracle.sweep(g.n, g.src, g.dst, g.w, np.array([e], np.int32), 1, x, L)
        assert float(np.dot(L, L)) <= q0 * (1 + 1e-15)


def test_limit_is_order_independent():
    """Fig. 1's caption and Property 2: the limit loads do not depend on the
    edge order."""
    rng = np.random.default_rng(12)
    g = synth.random_small(rng, 30, 0.25, True)
    _, _, order, _ = oracle.schedule(g.n, g.src, g.dst, 16)
    outs = []
    for o in (order, np.arange(g.m, dtype=np.int32), rng.permutation(g.m).astype(np.int32)):
        x, L = oracle.init(g.n, g.src, g.dst, g.w)
        oracle.sweep(g.n, g.src, g.dst, g.w, o, 5000, x, L)
        outs.append(L)
    assert np.allclose(outs[0], outs[1], atol=1e-8) and np.allclose(outs[0], outs[2], atol=1e-8)


def test_one_way_property_at_the_limit():
    """Property 3: at the optimum an edge between different loads gives all
    its weight to the lower endpoint."""
    g = graph_from_edges(9, [(0, 1), (0, 2), (1, 2), (0, 3), (1, 3), (2, 3), (3, 4), (4, 5),
                             (5, 6), (6, 7), (7, 8)])
    r = converge(g, 20000)
    L, x = r["L"], r["x"]
    for e in range(g.m):
        u, v = g.src[e], g.dst[e]
        if L[u] > L[v] + 1e-6:
            assert x[e] < 1e-9
        elif L[v] > L[u] + 1e-6:
            assert x[e] > 1 - 1e-9


# --------------------------------------------------------------- schedule --
def test_schedule_phases_are_star_forests():
    g = synth.workload(0)
    for smax in (1, 4, 16, 32):
        phase, center, order, P = oracle.schedule(g.n, g.src, g.dst, smax)
        assert np.array_equal(np.sort(order), np.arange(g.m))
        assert np.all(np.diff(phase[order]) >= 0)
        for p in range(P):
            es = np.flatnonzero(phase == p)
            c = center[es]
            l = np.where(g.src[es] == c, g.dst[es], g.src[es])
            # a leaf appears once and is never a center; centers have <= smax leaves
            assert np.unique(l).size == l.size
            assert not set(l.tolist()) & set(c.tolist())
            assert np.bincount(c).max() <= smax
        if smax == 1:
            # stars of one edge: the phases are matchings (proper edge colouring)
            deg = np.bincount(g.src, minlength=g.n) + np.bincount(g.dst, minlength=g.n)
            assert P >= deg.max()


def _splitmix64(k):
    """the k-th output (k = 1, 2, ...) of SplitMix64 seeded with 0"""
    M = (1 << 64) - 1
    z = (k * 0x9E3779B97F4A7C15) & M
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M
    return z ^ (z >> 31)


def test_splitmix64_known_answers():
    """The first outputs of SplitMix64 seeded with 0, as its reference
    implementation (Steele, Lea, Flood 2014; Vigna's splitmix64.c) prints."""
    assert [_splitmix64(k) for k in (1, 2, 3)] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4,
                                                   0x06C45D188009454F]


def test_schedule_first_fit_is_minimal():
    """Each edge sits in the first phase that admits it when the edges are
    visited by ascending SplitMix64 key (ties by index): moving it to any
    earlier phase would break the star-forest rule or the size limit."""
    rng = np.random.default_rng(2)
    g = synth.random_small(rng, 40, 0.3)
    smax = 3
    phase, center, order, P = oracle.schedule(g.n, g.src, g.dst, smax)
    deg = np.bincount(g.src, minlength=g.n) + np.bincount(g.dst, minlength=g.n)
    # the center is the endpoint of larger degree, ties to the smaller id
    exp_c = np.where((deg[g.src] > deg[g.dst]) | ((deg[g.src] == deg[g.dst]) & (g.src < g.dst)),
                     g.src, g.dst)
    assert np.array_equal(center, exp_c)
    visit = sorted(range(g.m), key=lambda e: (_splitmix64(e + 1), e))
    role = {}
    for e in visit:
        c = int(center[e])
        l = int(g.dst[e] if g.src[e] == c else g.src[e])
        for p in range(phase[e]):
            rc = role.get((c, p), 0)
            rl = role.get((l, p), 0)
            assert not ((rc == 0 or (rc != "leaf" and rc < smax)) and rl == 0)
        rc = role.get((c, phase[e]), 0)
        role[(c, int(phase[e]))] = rc + 1
        role[(l, int(phase[e]))] = "leaf"


def test_certificate_on_unit_weights():
    """Section III-B: on an unweighted graph, once D - rho < 1/(n(n-1)) the
    extracted set is densest."""
    rng = np.random.default_rng(31)
    for g in _random_graphs(10, 5, 10, False, 31):
        rho, S = brute_force_densest(g.n, g.src, g.dst)
        r = converge(g, 3000)
        n = g.n
        if r["D"] - r["rho"] < 1.0 / (n * (n - 1)):
            assert Fraction(r["num"], r["den"]) == rho


# ------------------------------------------------- LDD read-out (Problem 2) --
def _levels_from_readout(r):
    """nested sets B_1 .. B_L and lambda_j as exact fractions of f, k"""
    level = r["level"]
    sets, lams = [], []
    kp, fp = 0, Fraction(0)
    for j, (k, f) in enumerate(zip(r["k_end"], r["f_end"])):
        sets.append(frozenset(np.flatnonzero(level <= j).tolist()))
        fj = Fraction(f)
        lams.append((fj - fp) / (int(k) - kp))
        kp, fp = int(k), fj
    return sets, lams


@pytest.mark.parametrize("weighted", [False, True])
def test_ldd_readout_equals_brute_force_ldd(weighted):
    """Problem 2 / Property 2: the decomposition read from converged loads
    (prefixes of the descending load order, largest maximiser per level) is
    the locally-dense decomposition by its definition over all subsets: the
    same nested sets and the same lambda per level."""
    for g in _random_graphs(25, 4, 9, weighted, 21 + weighted):
        levels, lam = brute_force_ldd(g.n, g.src, g.dst, g.w)
        r = converge(g, 6000)
        ro = oracle.ldd(g.n, g.src, g.dst, g.w, r["L"])
        sets, lams = _levels_from_readout(ro)
        assert sets == levels, (g.src, g.dst, g.w)
        for a, b in zip(lams, [lam[min(B - (levels[i - 1] if i else frozenset()))]
                               for i, B in enumerate(levels)]):
            if weighted:
                assert abs(float(a) - float(b)) <= 1e-9 * max(1.0, abs(float(b)))
            else:
                assert a == b


def test_ldd_readout_closed_forms():
    """Two disjoint cliques K_6 and K_3 plus a pendant path: levels K_6
    (lambda 5/2), K_3 (lambda 1), then the path (n-1)/n-type tail."""
    edges = [(i, j) for i in range(6) for j in range(i + 1, 6)]
    edges += [(6 + i, 6 + j) for i in range(3) for j in range(i + 1, 3)]
    edges += [(9, 10), (10, 11)]
    g = graph_from_edges(12, edges)
    r = converge(g, 3000)
    ro = oracle.ldd(g.n, g.src, g.dst, None, r["L"])
    sets, lams = _levels_from_readout(ro)
    assert sets[0] == frozenset(range(6)) and lams[0] == Fraction(5, 2)
    assert sets[1] == frozenset(range(9)) and lams[1] == Fraction(1)
    assert sets[2] == frozenset(range(12)) and lams[2] == Fraction(2, 3)
    assert len(sets) == 3


@pytest.mark.parametrize("T", [0, 2, 5, 40])
def test_ldd_first_level_is_the_extracted_set(T):
    """At any iteration the read-out's first level is the extraction's set
    S* (the largest prefix of maximal density), with lambda_1 = rho(S*)."""
    rng = np.random.default_rng(T)
    for _ in range(6):
        g = synth.random_small(rng, int(rng.integers(20, 80)), float(rng.uniform(0.05, 0.3)))
        if g.m == 0:
            continue
        r = converge(g, T)
        ex = oracle.extract(g.n, g.src, g.dst, None, r["L"])
        ro = oracle.ldd(g.n, g.src, g.dst, None, r["L"])
        assert np.array_equal((ro["level"] == 0).astype(np.uint8), ex["in_set"])
        assert ro["k_end"][0] == ex["den"] and ro["f_end"][0] == ex["num"]
        assert ro["k_end"][-1] == g.n and ro["f_end"][-1] == g.m


def _densest_k_brute(n, edges, k):
    from itertools import combinations
    best = 0
    for S in combinations(range(n), k):
        s = set(S)
        best = max(best, sum(1 for a, b in edges if a in s and b in s))
    return Fraction(best, k)


def test_dks_bound_holds_and_is_tight_at_levels():
    """Corollary 1: for every k the densest k-subgraph has density at most the
    bound read from the decomposition, with equality when k = |B_j|."""
    for g in _random_graphs(12, 5, 9, False, 33):
        r = converge(g, 6000)
        ro = oracle.ldd(g.n, g.src, g.dst, None, r["L"])
        edges = list(zip(g.src.tolist(), g.dst.tolist()))
        for k in range(1, g.n + 1):
            exact = _densest_k_brute(g.n, edges, k)
            bound = oracle.dks_bound(ro["k_end"], ro["f_end"], k)
            assert float(exact) <= bound + 1e-12, (k, exact, bound)
            if k in set(int(v) for v in ro["k_end"]):
                assert abs(float(exact) - bound) <= 1e-12, (k, exact, bound)


@pytest.mark.parametrize("weighted", [False, True])
def test_qp_optimum_is_the_decomposition_value(weighted):
    """Section III-C / Property 2: the QP objective converges to
    sum_u lambda_u^2 of the locally-dense decomposition (brute force), the
    reference for the QP-error curve; the read-out's levels give the same
    value, sum_j lambda_j^2 |level j|."""
    for g in _random_graphs(15, 4, 9, weighted, 41 + weighted):
        _, lam = brute_force_ldd(g.n, g.src, g.dst, g.w)
        qstar = float(sum(v * v for v in lam))
        r = converge(g, 6000)
        assert abs(r["sumL2"] - qstar) <= 1e-7 * max(1.0, qstar)
        ro = oracle.ldd(g.n, g.src, g.dst, g.w, r["L"])
        ke = np.concatenate([[0], ro["k_end"]])
        fe = np.concatenate([[0.0], ro["f_end"]])
        lam_j = np.diff(fe) / np.diff(ke)
        assert abs(float(np.sum(lam_j ** 2 * np.diff(ke))) - qstar) <= 1e-9 * max(1.0, qstar)


# ------------------------------------------- weighted pruning (Algorithm 2) --
def _weighted_graphs(count, seed, nmin=8, nmax=40):
    rng = np.random.default_rng(seed)
    out = []
    while len(out) < count:
        g = synth.random_small(rng, int(rng.integers(nmin, nmax + 1)),
                               float(rng.uniform(0.08, 0.35)))
        if g.m == 0:
            continue
        g.w = rng.lognormal(0.0, 1.0, size=g.m).astype(np.float32)
        out.append(g)
    return out


@pytest.mark.parametrize("c", [1.0, 2.5, 0.375])
def test_weighted_prune_with_equal_weights_is_the_unweighted_prune(c):
    """Scaling every weight by the same c changes no comparison deg < rho:
    the weighted rounds keep exactly the unweighted mask."""
    rng = np.random.default_rng(int(c * 8))
    for _ in range(15):
        g = synth.random_small(rng, int(rng.integers(10, 60)), float(rng.uniform(0.05, 0.3)))
        keep_u, rounds_u, nh_u, mh_u = oracle.prune(g.n, g.src, g.dst)
        keep_w, rounds_w, nh_w, mh_w, _ = oracle.prune_weighted(
            g.n, g.src, g.dst, np.full(g.m, c, np.float32))
        assert np.array_equal(keep_u, keep_w) and (rounds_u, nh_u, mh_u) == (rounds_w, nh_w, mh_w)


def test_weighted_prune_keeps_the_densest_subgraph():
    """Theorem 4's argument with weighted degrees: every node of the maximal
    densest subgraph (brute force) has weighted degree >= rho* >= rho(H) in
    H, so it survives; rho(H) >= rho(G); every node of H has degree >= rho(H)."""
    for g in _weighted_graphs(20, 5, 6, 12):
        keep, rounds, nh, mh, WH = oracle.prune_weighted(g.n, g.src, g.dst, g.w)
        rho, S = brute_force_densest(g.n, g.src, g.dst, g.w)
        assert all(keep[u] for u in S)
        wf = [Fraction(float(x)) for x in g.w]
        assert WH / nh >= sum(wf, Fraction(0)) / g.n
        deg = [Fraction(0)] * g.n
        for e in range(g.m):
            if keep[g.src[e]] and keep[g.dst[e]]:
                deg[g.src[e]] += wf[e]
                deg[g.dst[e]] += wf[e]
        assert all(deg[u] * nh >= WH for u in range(g.n) if keep[u])


def test_weighted_prune_matches_weighted_greedy():
    """Theorem 5 with weighted degrees: greedy peeling (minimum weighted
    degree first) passes through H, its density does not decrease before,
    and the first decrease comes at H or later."""
    checked = 0
    for g in _weighted_graphs(30, 8):
        keep, _, nh, mh, WH = oracle.prune_weighted(g.n, g.src, g.dst, g.w)
        sizes, order = greedy_peel_weighted(g.n, g.src, g.dst, g.w)
        k = g.n - nh
        assert sizes[k] == (WH, nh)
        assert set(order[k:]) == set(np.flatnonzero(keep))
        dens = [W / N for W, N in sizes]
        assert all(dens[i + 1] >= dens[i] for i in range(k))
        checked += 1
    assert checked == 30


# ------------------------------------------------ greedy peeling (Algorithm 3) --
def test_greedy_order_equals_an_independent_heap_greedy():
    """The oracle's plain greedy (a full scan per step) removes the same nodes
    in the same order as a heap-based implementation, with the same |E(S)|
    after every removal."""
    rng = np.random.default_rng(71)
    for _ in range(25):
        g = synth.random_small(rng, int(rng.integers(2, 120)), float(rng.uniform(0.02, 0.4)))
        r = oracle.greedy(g.n, g.src, g.dst)
        sizes, order = greedy_peel(g.n, g.src, g.dst)
        assert r["order"].tolist() == order
        assert [int(v) for v in r["rem_m"][:-1]] == [M for M, _ in sizes[1:]]


def test_greedy_is_a_half_approximation_and_keeps_the_first_maximum():
    """Charikar: the greedy set has density at least rho*/2 (brute force);
    S* is the first (largest) remaining set of maximal density."""
    for g in _random_graphs(30, 4, 12, False, 73):
        r = oracle.greedy(g.n, g.src, g.dst)
        rho_star, _ = brute_force_densest(g.n, g.src, g.dst)
        rho = Fraction(r["num"], r["den"])
        assert 2 * rho >= rho_star
        dens = [Fraction(g.m, g.n)] + [Fraction(int(r["rem_m"][k]), g.n - k - 1)
                                       for k in range(g.n - 1)]
        assert rho == max(dens) and r["best_i"] == dens.index(max(dens))


def test_greedy_passes_through_the_pruned_graph():
    """Theorem 5 with the oracle's own greedy and prune: the first n - n_h
    removals are exactly the nodes Algorithm 2 removes."""
    rng = np.random.default_rng(79)
    for _ in range(30):
        g = synth.random_small(rng, int(rng.integers(8, 80)), float(rng.uniform(0.05, 0.3)))
        if g.m == 0:
            continue
        keep, _, nh, mh = oracle.prune(g.n, g.src, g.dst)
        r = oracle.greedy(g.n, g.src, g.dst)
        k = g.n - nh
        assert set(r["order"][:k].tolist()) == set(np.flatnonzero(keep == 0).tolist())
        assert (int(r["rem_m"][k - 1]) if k > 0 else g.m) == mh
