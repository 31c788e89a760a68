"""GPU parity: the HIP path through the C interface against the FP64 CPU
oracle on the same seeded inputs.

FP64 state: fractions, loads, the max load, the densest set and its exact
density must be bit-identical to the oracle's sequential loop in schedule
order (stronger than the 1e-9 relative gate).  FP32-compensated state: loads
within 1e-5 relative of the FP64 oracle.  Pruning: mask, rounds and sizes
bit-exact."""
import os

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2307_15969_amd as lowd  # noqa: E402


def log(msg):
    print(msg, flush=True)


SPLITS = {"auto": (None, None),            # cost model
          "all_lds": (0, None),             # every phase that fits runs from LDS
          "no_lds": (1 << 30, 1 << 30),     # whole-GPU launches only
          "all_mid": (1 << 30, 0),          # every phase in one workgroup, loads in memory
          "mid_lds": (None, 0)}             # middle tier then LDS tier


@pytest.fixture
def split(monkeypatch):
    def _set(name):
        tail, mid = SPLITS[name]
        for var, v in (("LOWD_TAIL_SPLIT", tail), ("LOWD_MID_SPLIT", mid)):
            if v is None:
                monkeypatch.delenv(var, raising=False)
            else:
                monkeypatch.setenv(var, str(v))
    return _set


def graphs_small():
    rng = np.random.default_rng(5)
    out = [("workload0", synth.workload(0))]
    out.append(("gnp_w", synth.random_small(rng, 300, 0.05, weighted=True)))
    g = synth.chung_lu(20000, 200000, 2.1, seed=3, planted=60, p_planted=0.3)
    out.append(("chunglu20k", g))
    gw = synth.chung_lu(15000, 120000, 2.1, seed=4, weights="lognormal")
    out.append(("chunglu15k_w", gw))
    return out


GRAPHS = graphs_small()


def oracle_run(g, T, smax):
    phase, center, order, P = oracle.schedule(g.n, g.src, g.dst, smax)
    x, L = oracle.init(g.n, g.src, g.dst, g.w)
    oracle.sweep(g.n, g.src, g.dst, g.w, order, T, x, L)
    return x, L, phase, center, P


def gpu_state(sv):
    x, L = sv.read_state()
    torch.cuda.synchronize()
    return x.cpu().numpy(), L.cpu().numpy()


@pytest.mark.parametrize("name,g", GRAPHS, ids=[n for n, _ in GRAPHS])
def test_init_is_bit_exact(name, g):
    log(f"init {name} n={g.n} m={g.m}")
    sv = lowd.Solver(g.n, g.src, g.dst, g.w, "f64")
    x, L = gpu_state(sv)
    xo, Lo = oracle.init(g.n, g.src, g.dst, g.w)
    assert np.array_equal(x, xo)
    assert np.array_equal(L, Lo)


@pytest.mark.parametrize("tier", list(SPLITS))
@pytest.mark.parametrize("smax", [1, 16, 32])
@pytest.mark.parametrize("name,g", GRAPHS, ids=[n for n, _ in GRAPHS])
def test_sweeps_are_bit_exact(name, g, smax, tier, split):
    split(tier)
    log(f"sweeps {name} smax={smax} tier={tier}")
    sv = lowd.Solver(g.n, g.src, g.dst, g.w, "f64", star_max=smax)
    info = sv.info()
    log(f"  info {info}")
    if tier == "no_lds":
        assert info["lds_phases"] == 0 and info["mid_phases"] == 0
    if tier == "all_mid":
        # phases with stars deeper than 16 leaves run as whole-GPU launches
        assert info["lds_phases"] == 0
        assert info["grid_phases"] == 0 or smax > 16
    T = 7
    # several launches of the sweep graph with eager work in between
    sv.iterate(1)
    sv.check()
    sv.iterate(2)
    sv.extract()
    sv.iterate(T - 3)
    x, L = gpu_state(sv)
    xo, Lo, phase, center, P = oracle_run(g, T, smax)
    assert info["phases"] == P
    assert np.array_equal(L, Lo), np.flatnonzero(L != Lo)[:10]
    assert np.array_equal(x, xo)
    D, s, s2 = sv.check()
    Do, so, s2o = oracle.stats(Lo)
    assert D == Do
    assert abs(s - so) <= 1e-12 * abs(so) and abs(s2 - s2o) <= 1e-12 * abs(s2o)


@pytest.mark.parametrize("tier", ["auto", "no_lds", "all_mid"])
def test_reset_restores_the_initial_state(tier, split):
    """A reset after some sweeps gives back Algorithm 1's initial state (the
    loads at every node's first station, the fractions), and the sweeps after
    it follow the oracle from there."""
    split(tier)
    g = GRAPHS[2][1]
    sv = lowd.Solver(g.n, g.src, g.dst, g.w, "f64")
    sv.iterate(3)
    sv.check()
    sv.reset()
    x, L = gpu_state(sv)
    xo, Lo = oracle.init(g.n, g.src, g.dst, g.w)
    assert np.array_equal(L, Lo) and np.array_equal(x, xo)
    sv.iterate(4)
    x, L = gpu_state(sv)
    xo, Lo, *_ = oracle_run(g, 4, 16)
    assert np.array_equal(L, Lo) and np.array_equal(x, xo)


@pytest.mark.parametrize("name,g", GRAPHS, ids=[n for n, _ in GRAPHS])
def test_schedule_export_equals_oracle(name, g):
    sv = lowd.Solver(g.n, g.src, g.dst, g.w, "f64", star_max=16)
    phase, center, P = sv.schedule()
    po, co, _, Po = oracle.schedule(g.n, g.src, g.dst, 16)
    assert P == Po and np.array_equal(phase, po) and np.array_equal(center, co)


@pytest.mark.parametrize("T", [0, 3, 40])
@pytest.mark.parametrize("name,g", GRAPHS, ids=[n for n, _ in GRAPHS])
def test_extraction_matches_oracle(name, g, T):
    log(f"extract {name} T={T}")
    sv = lowd.Solver(g.n, g.src, g.dst, g.w, "f64")
    sv.iterate(T)
    ex = sv.extract()
    xo, Lo, *_ = oracle_run(g, T, 16)
    ro = oracle.extract(g.n, g.src, g.dst, g.w, Lo)
    Do, _, _ = oracle.stats(Lo)
    assert ex["D"] == Do
    got = ex["in_set"].cpu().numpy()
    # densities are decided exactly on both sides (weights as exact integer
    # sums), so the set, |S| and W(S) (rounded once) are bit-identical
    assert np.array_equal(got, ro["in_set"])
    assert ex["den"] == ro["den"] and ex["num_w"] == ro["num_w"]
    if g.w is None:
        assert ex["num"] == ro["num"]


@pytest.mark.parametrize("T", [0, 2])
def test_extraction_with_several_sort_tiles_per_block(T):
    """300,001 nodes: the radix sort's blocks take two tiles each and the
    last block is partial; at T = 0 the loads are degree / 2, so many keys
    tie and the order among them is by node id.  Set and exact density equal
    the oracle's."""
    g = synth.chung_lu(300001, 1200000, 2.3, seed=9)
    log(f"n={g.n} m={g.m} T={T}")
    sv = lowd.Solver(g.n, g.src, g.dst, None, "f64")
    sv.iterate(T)
    ex = sv.extract()
    _, Lo, *_ = oracle_run(g, T, 16)
    ro = oracle.extract(g.n, g.src, g.dst, None, Lo)
    assert (ex["num"], ex["den"]) == (ro["num"], ro["den"])
    assert np.array_equal(ex["in_set"].cpu().numpy(), ro["in_set"])
    sv.close()


def test_workload0_reaches_the_maxflow_optimum():
    """200 sweeps on ER(1000, 5000) + K_30: the densest set and its exact
    density equal the oracle's, which max-flow certifies in the CPU pins."""
    g = synth.workload(0)
    sv = lowd.Solver(g.n, g.src, g.dst, None, "f64")
    sv.iterate(200)
    ex = sv.extract()
    ro = oracle.solve(g.n, g.src, g.dst, None, 200)
    assert (ex["num"], ex["den"]) == (ro["num"], ro["den"]) == (435, 30)
    assert np.array_equal(ex["in_set"].cpu().numpy(), ro["in_set"])


@pytest.mark.parametrize("name,g", GRAPHS, ids=[n for n, _ in GRAPHS])
def test_f32_compensated_within_tolerance(name, g):
    T = 25
    log(f"f32k {name}")
    sv = lowd.Solver(g.n, g.src, g.dst, g.w, "f32k")
    sv.iterate(T)
    x, L = gpu_state(sv)
    xo, Lo, *_ = oracle_run(g, T, 16)
    err = np.max(np.abs(L - Lo)) / np.max(np.abs(Lo))
    log(f"  max rel load error {err:.3e}")
    assert err <= 1e-5
    # D comes from FP64 loads recomputed from the FP32 fractions
    D, s, _ = sv.check()
    Do, so, _ = oracle.stats(Lo)
    assert abs(D - Do) <= 1e-5 * Do
    wsum = g.m if g.w is None else float(np.sum(g.w.astype(np.float64)))
    assert abs(s - wsum) <= 1e-9 * wsum


def _induced(g, in_set):
    """(W(S), |S|) of a node mask, counted on the CPU in FP64."""
    keep = in_set.astype(bool)
    both = keep[g.src] & keep[g.dst]
    num = float(np.sum(g.w.astype(np.float64)[both])) if g.w is not None else float(both.sum())
    return num, int(keep.sum())


@pytest.mark.parametrize("state", ["f64", "f32k"])
@pytest.mark.parametrize("name,g", GRAPHS, ids=[n for n, _ in GRAPHS])
def test_kept_check_and_extract(name, g, state):
    """The kept-load variants: for FP64 identical to the exact calls; for
    FP32K D within the FP32 load bound of the oracle's, and the extracted
    set's density exact for that set."""
    T = 25
    log(f"kept {name} {state}")
    sv = lowd.Solver(g.n, g.src, g.dst, g.w, state)
    sv.iterate(T)
    Dk, sk, s2k = sv.check(kept=True)
    D, s, s2 = sv.check()
    ek = sv.extract(kept=True)
    e = sv.extract()
    _, Lo, *_ = oracle_run(g, T, 16)
    Do, _, _ = oracle.stats(Lo)
    if state == "f64":
        assert (Dk, sk, s2k) == (D, s, s2)
        assert np.array_equal(ek["in_set"].cpu().numpy(), e["in_set"].cpu().numpy())
        assert (ek["num"], ek["num_w"], ek["den"], ek["D"]) == (e["num"], e["num_w"], e["den"], e["D"])
    else:
        assert abs(Dk - Do) <= 1e-5 * Do
        assert abs(ek["D"] - Do) <= 1e-5 * Do
    num, den = _induced(g, ek["in_set"].cpu().numpy())
    assert den == ek["den"]
    got = ek["num"] if g.w is None else ek["num_w"]
    assert abs(got - num) <= 1e-12 * max(num, 1.0)


@pytest.mark.parametrize("name,g", GRAPHS, ids=[n for n, _ in GRAPHS])
def test_f32k_resync_restarts_from_the_fractions_loads(name, g):
    """After a resync the carried FP32K loads are the loads recomputed from
    the fractions (to the precision of the (s, c) pair), the fractions are
    untouched, and further sweeps stay within the FP32 tolerance of the
    oracle; for FP64 a resync changes nothing."""
    T = 15
    for state in ("f32k", "f64"):
        sv = lowd.Solver(g.n, g.src, g.dst, g.w, state)
        sv.iterate(T)
        x0, L0 = (t.cpu().numpy() for t in sv.read_state())
        D = sv.check()[0]
        sv.resync()
        x1, L1 = (t.cpu().numpy() for t in sv.read_state())
        assert np.array_equal(x0, x1)
        Dk = sv.check(kept=True)[0]
        if state == "f64":
            assert np.array_equal(L0, L1) and Dk == D
        else:
            assert abs(Dk - D) <= 1e-13 * max(D, 1.0)
            sv.iterate(T)
            _, Lo, *_ = oracle_run(g, 2 * T, 16)
            _, L2 = sv.read_state()
            L2 = L2.cpu().numpy()
            assert np.max(np.abs(L2 - Lo)) <= 1e-5 * np.max(np.abs(Lo))
        sv.close()


def test_f32k_solve_certifies_with_the_exact_bound():
    """solve() screens with the kept FP32K loads but returns a gap taken
    from the exact D (recomputed from the fractions), and its set is as
    dense as the FP64 solve's within the tolerance."""
    g = GRAPHS[2][1]
    tol = 1e-6
    r32 = lowd.solve(g.n, g.src, g.dst, g.w, "f32k", tol=tol)
    r64 = lowd.solve(g.n, g.src, g.dst, g.w, "f64", tol=tol)
    D = r32["solver"].check()[0]
    assert r32["D"] == D
    rho32 = r32["num"] / r32["den"]
    rho64 = r64["num"] / r64["den"]
    assert (D - rho32) / rho32 <= tol and r32["gap"] <= tol
    assert abs(rho32 - rho64) <= 2 * tol * rho64
    log(f"  f32k {r32['sweeps']} sweeps, f64 {r64['sweeps']} sweeps")


def test_unit_graph_f32k_finds_the_same_densest_set():
    g = synth.workload(0)
    sv = lowd.Solver(g.n, g.src, g.dst, None, "f32k")
    sv.iterate(200)
    ex = sv.extract()
    assert (ex["num"], ex["den"]) == (435, 30)


# ---------------------------------------------------------------- pruning --
PRUNE_GRAPHS = [("workload0", synth.workload(0)),
                ("chunglu20k", GRAPHS[2][1]),
                ("gnp", synth.random_small(np.random.default_rng(1), 400, 0.03)),
                ("empty", synth.canonical(7, np.zeros(0, np.int64), np.zeros(0, np.int64))),
                ("one_edge", synth.canonical(3, np.array([2]), np.array([0]))),
                ("star", synth.canonical(5000, np.zeros(4999, np.int64), np.arange(1, 5000))),
                ("rmat14", synth.rmat(14, 16, seed=2))]


@pytest.mark.parametrize("name,g", PRUNE_GRAPHS, ids=[n for n, _ in PRUNE_GRAPHS])
def test_prune_matches_oracle(name, g):
    log(f"prune {name} n={g.n} m={g.m}")
    r = lowd.prune(g.n, g.src, g.dst)
    keep, rounds, nh, mh = oracle.prune(g.n, g.src, g.dst)
    assert np.array_equal(r["node_keep"].cpu().numpy(), keep)
    assert (r["rounds"], r["n_h"], r["m_h"]) == (rounds, nh, mh)
    relabel = np.cumsum(keep.astype(np.int64)) - 1
    relabel[keep == 0] = -1
    assert np.array_equal(r["relabel"].cpu().numpy(), relabel)
    ek = (keep[g.src] == 1) & (keep[g.dst] == 1)
    assert np.array_equal(r["edge_map"].cpu().numpy(), np.flatnonzero(ek))
    assert np.array_equal(r["src"].cpu().numpy(), relabel[g.src[ek]])
    assert np.array_equal(r["dst"].cpu().numpy(), relabel[g.dst[ek]])


def test_prune_with_sorts_large_enough_to_stage():
    """R-MAT scale 19 (about 7M edges): the incidence sort (14M keys) takes
    the radix sort's LDS-staged scatter, the pair sort of the validation the
    per-tile one; the pruned graph equals the oracle's."""
    g = synth.rmat(19, 16, seed=5)
    log(f"n={g.n} m={g.m}")
    assert 2 * g.m > 32 * 1024 * 256
    r = lowd.prune(g.n, g.src, g.dst)
    keep, rounds, nh, mh = oracle.prune(g.n, g.src, g.dst)
    assert np.array_equal(r["node_keep"].cpu().numpy(), keep)
    assert (r["rounds"], r["n_h"], r["m_h"]) == (rounds, nh, mh)
    ek = (keep[g.src] == 1) & (keep[g.dst] == 1)
    assert np.array_equal(r["edge_map"].cpu().numpy(), np.flatnonzero(ek))


def _degree_count_shapes():
    rng = np.random.default_rng(7)

    def skewed(n, ids, k, power):
        p = 1.0 / np.arange(1, ids.size + 1) ** power
        p /= p.sum()
        return synth.canonical(n, ids[rng.choice(ids.size, k, p=p)],
                               ids[rng.choice(ids.size, k, p=p)])

    # node ids of 25 bits: the ends are grouped by their top 8 bits and each
    # group is counted in four id ranges of 32K
    n1 = (1 << 24) + (1 << 22)
    wide = skewed(n1, rng.choice(n1, 400_000, replace=False), 1_500_000, 0.8)
    # 32,768 nodes (ids of 15 bits: one group) and over 4M ends: the group
    # is counted in pieces whose counts are added
    dense = skewed(1 << 15, rng.permutation(1 << 15), 3_000_000, 0.8)
    # 8,192 core nodes and 24,576 others joined to about 400 core nodes each:
    # the first round removes the others, and the degrees lost by the core
    # nodes outside the 4,096 hubs (about 4.7M) are taken off in pieces
    r2 = np.random.default_rng(11)
    n3, core = 1 << 15, 8192
    per = np.repeat(np.arange(core, n3), 400)
    pieces = synth.canonical(
        n3, np.concatenate([r2.integers(0, core, 4_200_000), per]),
        np.concatenate([r2.integers(0, core, 4_200_000), r2.integers(0, core, per.size)]))
    return [("wide_ids", wide), ("dense_pieces", dense), ("decrement_pieces", pieces)]


@pytest.mark.parametrize("name,g", _degree_count_shapes(),
                         ids=["wide_ids", "dense_pieces", "decrement_pieces"])
def test_prune_degree_count_shapes(name, g):
    """The degree count's uncommon shapes: node ids wider than 24 bits
    (several id ranges per group), a group with more ends than one workgroup
    counts (pieces added with atomics), and a round whose decrements need
    such pieces (taken off with atomics); the pruned graph equals the
    oracle's."""
    log(f"prune {name} n={g.n} m={g.m}")
    assert 2 * g.m > (1 << 22) or g.n > (1 << 24)
    r = lowd.prune(g.n, g.src, g.dst)
    keep, rounds, nh, mh = oracle.prune(g.n, g.src, g.dst)
    assert (r["rounds"], r["n_h"], r["m_h"]) == (rounds, nh, mh)
    assert np.array_equal(r["node_keep"].cpu().numpy(), keep)
    assert rounds >= 1 and 0 < nh < g.n
    ek = (keep[g.src] == 1) & (keep[g.dst] == 1)
    assert np.array_equal(r["edge_map"].cpu().numpy(), np.flatnonzero(ek))


def test_prune_then_solve_finds_the_densest_set_of_g():
    g = synth.workload(0)
    r = lowd.prune(g.n, g.src, g.dst)
    sv = lowd.Solver(r["n_h"], r["src"], r["dst"], None, "f64")
    sv.iterate(200)
    ex = sv.extract()
    in_h = ex["in_set"].cpu().numpy().astype(bool)
    kept = np.flatnonzero(r["node_keep"].cpu().numpy())
    ro = oracle.solve(g.n, g.src, g.dst, None, 200)
    assert set(kept[in_h].tolist()) == set(np.flatnonzero(ro["in_set"]).tolist())
    assert (ex["num"], ex["den"]) == (ro["num"], ro["den"])


def test_entry_points_on_a_side_stream():
    """Every call orders its copies on the caller's stream: on a torch side
    stream (created non-blocking, so it does not wait for the null stream)
    the prune, the check of the edge list, greedy and the solve give the
    oracle's results, and a repeated pair is still named."""
    g = PRUNE_GRAPHS[4][1]
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        r = lowd.prune(g.n, g.src, g.dst)
        keep = r["node_keep"].cpu().numpy()
        gr = lowd.greedy_peel(g.n, g.src, g.dst)
        sv = lowd.solve(g.n, g.src, g.dst, None, state="f64", tol=1e-9)
        src = np.concatenate([g.src, g.src[:1]])
        dst = np.concatenate([g.dst, g.dst[:1]])
        with pytest.raises(RuntimeError, match=f"at index {g.m}:"):
            lowd.prune(g.n, src, dst)
    side.synchronize()
    ko, rounds, nh, mh = oracle.prune(g.n, g.src, g.dst)
    assert np.array_equal(keep, ko)
    assert (r["rounds"], r["n_h"], r["m_h"]) == (rounds, nh, mh)
    go = oracle.greedy(g.n, g.src, g.dst)
    assert np.array_equal(gr["order"].cpu().numpy(), go["order"])
    assert (gr["num"], gr["den"]) == (go["num"], go["den"])
    assert sv["gap"] <= 1e-9


# ------------------------------------------------------------ edge cases --
def test_graph_without_edges():
    g = synth.canonical(5, np.zeros(0, np.int64), np.zeros(0, np.int64))
    sv = lowd.Solver(5, g.src, g.dst, None, "f64")
    sv.iterate(3)
    x, L = gpu_state(sv)
    assert np.all(L == 0)
    ex = sv.extract()
    assert ex["den"] == 5 and ex["num"] == 0


def test_single_edge_and_isolated_nodes():
    g = synth.canonical(6, np.array([4]), np.array([1]))
    sv = lowd.Solver(6, g.src, g.dst, None, "f64")
    sv.iterate(4)
    x, L = gpu_state(sv)
    assert L.tolist() == [0, 0.5, 0, 0, 0.5, 0]
    ex = sv.extract()
    assert (ex["num"], ex["den"]) == (1, 2)
    assert ex["in_set"].cpu().numpy().tolist() == [0, 1, 0, 0, 1, 0]


def test_single_node():
    sv = lowd.Solver(1, np.zeros(0, np.int32), np.zeros(0, np.int32), None, "f64")
    ex = sv.extract()
    assert ex["den"] == 1


def test_degenerate_graphs_for_every_entry_point():
    """No edges, one node, one edge: the decomposition read-out, the trace,
    greedy peeling and both prunes give the definitions' answers."""
    empty = synth.canonical(5, np.zeros(0, np.int64), np.zeros(0, np.int64))
    one = synth.canonical(1, np.zeros(0, np.int64), np.zeros(0, np.int64))
    edge = synth.canonical(6, np.array([4]), np.array([1]))
    for g in (empty, one, edge):
        sv = lowd.Solver(g.n, g.src, g.dst, None, "f64")
        r = sv.ldd()
        ro = oracle.ldd(g.n, g.src, g.dst, None, oracle_run(g, 0, 16)[1])
        assert np.array_equal(r["k_end"], ro["k_end"]) and np.array_equal(r["f_end"], ro["f_end"])
        assert np.array_equal(r["level"].cpu().numpy(), ro["level"])
        tr = sv.trace(0, 3)
        assert tr.shape == (1, 5) and tr[0, 0] == 0
        gr = lowd.greedy_peel(g.n, g.src, g.dst)
        go = oracle.greedy(g.n, g.src, g.dst)
        assert np.array_equal(gr["order"].cpu().numpy(), go["order"])
        assert (gr["num"], gr["den"]) == (go["num"], go["den"])
        pu = lowd.prune(g.n, g.src, g.dst)
        pw = lowd.prune_weighted(g.n, g.src, g.dst, np.ones(g.m, np.float32))
        ko, rounds, nh, mh = oracle.prune(g.n, g.src, g.dst)
        for p_ in (pu, pw):
            assert np.array_equal(p_["node_keep"].cpu().numpy(), ko)
            assert (p_["n_h"], p_["m_h"]) == (nh, mh)
        sv.close()
    # the kept-load calls and the resync, in both states
    for g in (empty, one, edge):
        for state in ("f64", "f32k"):
            sv = lowd.Solver(g.n, g.src, g.dst, None, state)
            sv.iterate(3)
            assert sv.check(kept=True) == sv.check()
            ek, e = sv.extract(kept=True), sv.extract()
            assert (ek["num"], ek["den"], ek["D"]) == (e["num"], e["den"], e["D"])
            sv.resync()
            assert sv.check() == sv.check(kept=True)
            r = lowd.solve(g.n, g.src, g.dst, None, state)
            assert r["gap"] <= 1e-6 and (r["num"], r["den"]) == (e["num"], e["den"])
            sv.close()
    # the single edge: one level of density 1/2, then the isolated nodes at 0
    sv = lowd.Solver(edge.n, edge.src, edge.dst, None, "f64")
    sv.iterate(2)
    r = sv.ldd()
    assert r["k_end"].tolist() == [2, 6] and r["f_end"].tolist() == [1.0, 1.0]
    assert lowd.dks_bound(r["k_end"], r["f_end"], 1) == 0.5


def test_batch_degenerate_graphs_and_tiny_batches():
    """A batch of one graph; graphs without edges retire at once; an
    all-converged batch iterates nothing."""
    gs = [synth.canonical(3, np.zeros(0, np.int64), np.zeros(0, np.int64)),
          synth.canonical(2, np.array([0]), np.array([1]))]
    b = lowd.Batch(gs, "f64")
    b.iterate(3)
    b.extract(loads=True)
    assert b.load.cpu().numpy().tolist() == [0, 0, 0, 0.5, 0.5]
    assert b.num.cpu().numpy().tolist() == [0, 1] and b.den.cpu().numpy().tolist() == [3, 2]
    active, edges = b.retire(0.0)
    assert (active, edges) == (0, 0)
    b.iterate(5)            # nothing left to sweep
    b.extract(loads=True)
    assert b.load.cpu().numpy().tolist() == [0, 0, 0, 0.5, 0.5]
    b.close()
    single = lowd.Batch([synth.workload(0)], "f64", tune=True)
    single.iterate(4)
    single.extract(loads=True)
    xo, Lo, *_ = oracle_run(synth.workload(0), 4, 16)
    assert np.array_equal(single.load.cpu().numpy(), Lo)
    single.close()


@pytest.mark.parametrize("src,dst,w,what", [
    ([0, 2], [1, 2], None, "self-loop"),
    ([0, 1], [1, 9], None, "out of range"),
    ([0, 1, 0], [1, 2, 1], None, "repeated"),
    ([0, 1], [1, 2], [1.0, 0.0], "zero weight"),
    ([0, 1], [1, 2], [1.0, float("nan")], "nan weight"),
    ([0, 1], [1, 2], [1.0, -2.0], "negative weight"),
    ([0, 2], [1, 1], None, "reversed duplicate is fine"),
    ([3], [3], None, "single self-loop"),
    ([0], [7], None, "single out of range"),
    ([0, 0, 1], [1, 1, 1], None, "repeated pair before a self-loop"),
])
def test_invalid_graphs_are_rejected(src, dst, w, what):
    """Every kind of invalid edge list is rejected, and the message names the
    first invalid edge ahead of any repeated pair."""
    args = (5, np.array(src, np.int32), np.array(dst, np.int32),
            None if w is None else np.array(w, np.float32))
    if what.endswith("fine"):
        lowd.Solver(*args)
        return
    with pytest.raises(lowd.LowdError) as ei:
        lowd.Solver(*args)
    assert ei.value.status == -2, what
    kind = "repeated pair" if what == "repeated" else "invalid edge"
    assert kind in str(ei.value), (what, str(ei.value))
    if what == "repeated pair before a self-loop":
        assert "at index 2:" in str(ei.value)


def test_repeated_pair_in_reverse_orientation_is_rejected():
    with pytest.raises(lowd.LowdError) as ei:
        lowd.Solver(4, np.array([0, 1], np.int32), np.array([1, 0], np.int32))
    assert ei.value.status == -2


@pytest.mark.parametrize("copies", [2, 9000])
def test_repeated_pair_is_named_by_its_first_repeat(copies):
    """A pair repeated among many distinct edges is rejected, and the message
    names the first edge whose pair appeared before.  9,000 copies of one
    pair overflow its hash bucket, so the check falls back to the full sort
    of the pairs (a0: no repeated unordered pair)."""
    rng = np.random.default_rng(copies)
    n = 1 << 16
    a = rng.integers(0, n, 600000)
    b = rng.integers(0, n, 600000)
    keep = a != b
    lo, hi = np.minimum(a, b)[keep], np.maximum(a, b)[keep]
    key = np.unique(lo.astype(np.int64) * n + hi)
    src, dst = (key // n).astype(np.int32), (key % n).astype(np.int32)
    perm = rng.permutation(src.size)
    src, dst = src[perm], dst[perm]
    rep = np.full(copies, 7, np.int32), np.full(copies, 11, np.int32)
    pos = src.size // 3
    src = np.concatenate([src[:pos], rep[0], src[pos:]]).astype(np.int32)
    dst = np.concatenate([dst[:pos], rep[1], dst[pos:]]).astype(np.int32)
    # flip the orientation of every other copy
    dst[pos + 1:pos + copies:2], src[pos + 1:pos + copies:2] = 7, 11
    pair = np.minimum(src, dst).astype(np.int64) * n + np.maximum(src, dst)
    _, first = np.unique(pair, return_index=True)
    seen = np.zeros(src.size, bool)
    seen[first] = True
    expect = int(np.flatnonzero(~seen)[0])
    log(f"m={src.size} copies={copies} first repeat at {expect}")
    for call in (lambda: lowd.Solver(n, src, dst), lambda: lowd.prune(n, src, dst)):
        with pytest.raises(lowd.LowdError) as ei:
            call()
        assert ei.value.status == -2
        assert f"at index {expect}:" in str(ei.value), str(ei.value)


def _first_repeat(src, dst, n):
    pair = np.minimum(src, dst).astype(np.int64) * n + np.maximum(src, dst)
    _, first = np.unique(pair, return_index=True)
    seen = np.zeros(src.size, bool)
    seen[first] = True
    return int(np.flatnonzero(~seen)[0])


@pytest.mark.parametrize("where", ["hub_row", "hub_pair", "short_rows"])
def test_prune_finds_a_repeated_pair_in_every_kind_of_row(where):
    """A repeated pair is found by the prune's check of its edge list and
    named by its first repeat, whether its smaller end is a hub of 3,000
    neighbours (hub_row), both ends are (hub_pair), or neither (short_rows:
    repeats planted at random places of an R-MAT edge list, in either
    orientation); the same graph without the repeat prunes as the oracle
    does."""
    rng = np.random.default_rng(7)
    n = 1 << 14
    if where in ("hub_row", "hub_pair"):
        g = synth.rmat(14, 16, seed=3)
        src, dst = g.src.astype(np.int32), g.dst.astype(np.int32)
        hub, hub2 = 5, 9
        # two hubs of 3,000 neighbours each (pairs not yet in the graph)
        have = set((np.minimum(src, dst).astype(np.int64) * n + np.maximum(src, dst)).tolist())
        extra_s, extra_d = [], []
        for h in (hub, hub2):
            added = 0
            for v in rng.permutation(n)[:6000].tolist():
                if added == 3000:
                    break
                a, b = min(h, v), max(h, v)
                if v != h and a * n + b not in have:
                    have.add(a * n + b)
                    extra_s.append(h)
                    extra_d.append(v)
                    added += 1
        if hub * n + hub2 not in have:
            extra_s.append(hub)
            extra_d.append(hub2)
        src = np.concatenate([src, np.array(extra_s, np.int32)])
        dst = np.concatenate([dst, np.array(extra_d, np.int32)])
        perm = rng.permutation(src.size)
        src, dst = src[perm], dst[perm]
        # no repeat yet: the prune runs and equals the oracle's
        r = lowd.prune(n, src, dst)
        keep, rounds, nh, mh = oracle.prune(n, src, dst)
        assert np.array_equal(r["node_keep"].cpu().numpy(), keep) and r["m_h"] == mh
        pair = (hub, int(extra_d[len(extra_d) // 3])) if where == "hub_row" else (hub2, hub)
        cases = [pair]
    else:
        g = synth.rmat(14, 16, seed=4)
        src, dst = g.src.astype(np.int32), g.dst.astype(np.int32)
        cases = []
        for k in range(4):
            e = int(rng.integers(0, src.size))
            cases.append((int(src[e]), int(dst[e])))
    for a, b in cases:
        pos = int(rng.integers(0, src.size + 1))
        flip = bool(rng.integers(0, 2))
        s2 = np.insert(src, pos, b if flip else a).astype(np.int32)
        d2 = np.insert(dst, pos, a if flip else b).astype(np.int32)
        expect = _first_repeat(s2, d2, n)
        log(f"{where}: pair ({a}, {b}) again at {pos}, first repeat {expect}")
        with pytest.raises(lowd.LowdError) as ei:
            lowd.prune(n, s2, d2)
        assert ei.value.status == -2
        assert f"at index {expect}:" in str(ei.value), str(ei.value)


# ------------------------------------------------- full-size workload ----
def test_chunglu_1m_10m_fp64_is_bit_exact():
    """The benchmark workload at full size (Chung-Lu n=1M, ~10M edges,
    beta=2.1, planted 500-node block of density 0.3), in the launch
    configuration the benchmark times: 3 sweeps, loads, fractions and
    densest set identical to the oracle."""
    g = synth.workload(1, seed=1)
    log(f"workload1 n={g.n} m={g.m}")
    sv = lowd.Solver(g.n, g.src, g.dst, None, "f64")
    log(f"  info {sv.info()}")
    T = 3
    sv.iterate(T)
    x, L = gpu_state(sv)
    ex = sv.extract()
    xo, Lo, phase, center, P = oracle_run(g, T, 16)
    assert np.array_equal(L, Lo)
    assert np.array_equal(x, xo)
    ro = oracle.extract(g.n, g.src, g.dst, None, Lo)
    assert (ex["num"], ex["den"]) == (ro["num"], ro["den"])
    assert np.array_equal(ex["in_set"].cpu().numpy(), ro["in_set"])


def _digest(a) -> str:
    import hashlib
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def test_rmat24_full_size_prune_and_three_sweeps():
    """The headline workload at full size, in the benchmark's configuration:
    R-MAT scale 24 (260M edges) pruned on the GPU, then the FP64 solver on H
    with stars of at most 32 leaves, three sweeps.  The prune's rounds,
    sizes and mask, the loads and fractions after three sweeps and the
    densest prefix equal the oracle's, bit for bit (digests of the oracle's
    results, written by tests/golden/make_rmat24_h.py from synth and the
    oracle alone: its sequential schedule takes minutes at this size)."""
    import json
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "rmat24_h.json")))
    g = synth.rmat(24, 16, seed=1, device="cuda")
    log(f"rmat24 n={g.n} m={g.m}")
    src = torch.from_numpy(g.src).cuda()
    dst = torch.from_numpy(g.dst).cuda()
    del g
    r = lowd.prune(1 << 24, src, dst)
    gp = gold["prune"]
    assert (r["rounds"], r["n_h"], r["m_h"]) == (gp["rounds"], gp["n_h"], gp["m_h"])
    assert _digest(r["node_keep"].cpu().numpy()) == gp["node_keep_sha256"]
    hs, hd = r["src"].clone(), r["dst"].clone()
    del r, src, dst
    sv = lowd.Solver(gp["n_h"], hs, hd, None, "f64", star_max=gold["star_max"])
    log(f"  H {gp['n_h']} / {gp['m_h']}, {sv.info()['phases']} phases")
    assert sv.info()["phases"] == gold["phases"]
    sv.iterate(gold["sweeps"])
    x, L = gpu_state(sv)
    assert _digest(L) == gold["loads_sha256"]
    assert _digest(x) == gold["fractions_sha256"]
    ex = sv.extract()
    ge = gold["extract"]
    assert (ex["num"], ex["den"]) == (ge["num"], ge["den"])
    assert _digest(ex["in_set"].cpu().numpy().astype(np.uint8)) == ge["in_set_sha256"]
    # the benchmark's solve (lowd_solve to a certified 1e-6 gap) stops after
    # those three sweeps with that set
    sv.reset()
    r = sv.solve(1e-6)
    assert r["converged"] and r["gap"] <= 1e-6 and r["sweeps"] == gold["sweeps"]
    assert (r["num"], r["den"]) == (ge["num"], ge["den"])
    assert _digest(r["in_set"].cpu().numpy().astype(np.uint8)) == ge["in_set_sha256"]


def test_chunglu4m_full_size_fp64_and_f32k():
    """The FP32-compensated workload at full size (Chung-Lu n=4M, about 63M
    log-normal weights, stars of at most 16 leaves), 22 sweeps as the
    benchmark's solve takes: the FP64 path's loads and fractions equal the
    oracle's bit for bit; the FP32K path's loads lie within 1e-5 of the
    largest load on 4,096 nodes (the 2,048 largest and 2,048 drawn), its D
    from the recomputed loads within 1e-5 and its load sum within 1e-9 of
    the oracle's; both give the oracle's densest prefix (digests and exact
    values from tests/golden/make_chunglu4m.py: synth and the oracle
    alone)."""
    import json
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "chunglu4m.json")))
    g = synth.workload(2, seed=1)
    log(f"chunglu4m n={g.n} m={g.m}")
    assert (g.n, g.m) == (gold["n"], gold["m"])
    src = torch.from_numpy(g.src).cuda()
    dst = torch.from_numpy(g.dst).cuda()
    w = torch.from_numpy(g.w).cuda()
    nodes = np.array(gold["sample_nodes"], dtype=np.int64)
    lo = np.array([float.fromhex(v) for v in gold["sample_loads"]])
    Do, so = float.fromhex(gold["D"]), float.fromhex(gold["load_sum"])
    ge = gold["extract"]
    T = gold["sweeps"]
    for state in ("f64", "f32k"):
        sv = lowd.Solver(g.n, src, dst, w, state, star_max=gold["star_max"])
        assert sv.info()["phases"] == gold["phases"]
        sv.iterate(T)
        x, L = gpu_state(sv)
        if state == "f64":
            assert _digest(L) == gold["loads_sha256"]
            assert _digest(x) == gold["fractions_sha256"]
        else:
            err = np.max(np.abs(L[nodes] - lo)) / Do
            log(f"  f32k: max load error on the sample {err:.3e} of the largest load")
            assert err <= 1e-5
            D, s, _ = sv.check()
            assert abs(D - Do) <= 1e-5 * Do
            assert abs(s - so) <= 1e-9 * so
        ex = sv.extract()
        log(f"  {state}: densest prefix {ex['num_w']}/{ex['den']}")
        assert (ex["num"], ex["den"]) == (ge["num"], ge["den"])
        assert ex["num_w"] == float.fromhex(ge["num_w"])
        assert _digest(ex["in_set"].cpu().numpy().astype(np.uint8)) == ge["in_set_sha256"]
        # the benchmark's solve to a certified 1e-6 gap ends on the same set
        sv.reset()
        r = sv.solve(1e-6)
        sv.close()
        log(f"  {state}: solve {r['sweeps']} sweeps, gap {r['gap']:.2e}")
        assert r["converged"] and r["gap"] <= 1e-6
        if state == "f64":
            assert r["sweeps"] == T
        assert (r["num"], r["den"], r["num_w"]) == (ge["num"], ge["den"], float.fromhex(ge["num_w"]))
        assert _digest(r["in_set"].cpu().numpy().astype(np.uint8)) == ge["in_set_sha256"]


# ------------------------------------------------- weighted pruning --
def _weighted_prune_graphs():
    rng = np.random.default_rng(17)
    out = []
    for i in range(6):
        g = synth.random_small(rng, int(rng.integers(30, 300)), float(rng.uniform(0.02, 0.2)))
        g.w = rng.lognormal(0.0, 1.0, size=g.m).astype(np.float32)
        out.append((f"gnp{i}", g))
    out.append(("chunglu15k_w", synth.chung_lu(15000, 120000, 2.1, seed=4, weights="lognormal")))
    return out


@pytest.mark.parametrize("name,g", _weighted_prune_graphs(), ids=lambda v: v if isinstance(v, str) else "")
def test_weighted_prune_matches_exact_oracle(name, g):
    """Algorithm 2 with weighted degrees: mask, rounds, sizes and the
    relabelled H (with weights) equal the exact rational oracle; w(E(H)) is
    the exact value rounded once."""
    log(f"weighted prune {name} n={g.n} m={g.m}")
    r = lowd.prune_weighted(g.n, g.src, g.dst, g.w)
    keep, rounds, nh, mh, WH = oracle.prune_weighted(g.n, g.src, g.dst, g.w)
    log(f"  rounds {r['rounds']} H {r['n_h']}/{r['m_h']}")
    assert np.array_equal(r["node_keep"].cpu().numpy(), keep)
    assert (r["rounds"], r["n_h"], r["m_h"]) == (rounds, nh, mh)
    assert r["w_h"] == float(WH)
    kept = np.flatnonzero(keep[g.src] & keep[g.dst])
    newid = np.cumsum(keep) - 1
    assert np.array_equal(r["edge_map"].cpu().numpy(), kept)
    assert np.array_equal(r["src"].cpu().numpy(), newid[g.src[kept]])
    assert np.array_equal(r["dst"].cpu().numpy(), newid[g.dst[kept]])
    assert np.array_equal(r["w"].cpu().numpy(), g.w[kept])


def test_weighted_prune_equal_weights_is_unweighted_prune():
    g = synth.chung_lu(20000, 200000, 2.1, seed=3, planted=60, p_planted=0.3)
    r = lowd.prune_weighted(g.n, g.src, g.dst, np.full(g.m, 0.75, np.float32))
    u = lowd.prune(g.n, g.src, g.dst)
    assert np.array_equal(r["node_keep"].cpu().numpy(), u["node_keep"].cpu().numpy())
    assert (r["rounds"], r["n_h"], r["m_h"]) == (u["rounds"], u["n_h"], u["m_h"])
    assert r["w_h"] == 0.75 * u["m_h"]


def test_weighted_prune_rejects_too_wide_a_weight_range():
    g = synth.canonical(4, np.array([0, 1, 2]), np.array([1, 2, 3]),
                        np.array([1.0, 2.0 ** -30, 2.0 ** 20], np.float32))
    with pytest.raises(lowd.LowdError) as ei:
        lowd.prune_weighted(g.n, g.src, g.dst, g.w)
    assert ei.value.status == -5


def test_weighted_prune_then_solve_keeps_the_optimum():
    """The densest set of G (weighted) lies in H: solving H and G to a 1e-7
    gap gives overlapping certified intervals [rho, D]."""
    g = synth.chung_lu(15000, 120000, 2.1, seed=4, weights="lognormal")
    r = lowd.prune_weighted(g.n, g.src, g.dst, g.w)
    eh = lowd.solve(r["n_h"], r["src"], r["dst"], r["w"], "f64", tol=1e-7)
    eg = lowd.solve(g.n, g.src, g.dst, g.w, "f64", tol=1e-7)
    rh = eh["num_w"] / eh["den"]
    rg = eg["num_w"] / eg["den"]
    log(f"  H: rho {rh} D {eh['D']}  G: rho {rg} D {eg['D']}")
    assert max(rh, rg) <= min(eh["D"], eg["D"]) * (1 + 1e-12)


# ---------------------------------------- greedy peeling plug-in (Alg. 3) --
def _greedy_graphs():
    rng = np.random.default_rng(23)
    out = [("workload0", synth.workload(0))]
    for i in range(4):
        out.append((f"gnp{i}", synth.random_small(rng, int(rng.integers(2, 400)),
                                                  float(rng.uniform(0.01, 0.3)))))
    out.append(("chunglu20k", synth.chung_lu(20000, 200000, 2.1, seed=3, planted=60,
                                             p_planted=0.3)))
    return out


@pytest.mark.parametrize("name,g", _greedy_graphs(), ids=lambda v: v if isinstance(v, str) else "")
def test_greedy_peel_matches_oracle(name, g):
    """Algorithm 3 on the GPU equals the oracle's sequential greedy: the
    removal order, |E(S)| after every removal, S* and its density."""
    log(f"greedy {name} n={g.n} m={g.m}")
    r = lowd.greedy_peel(g.n, g.src, g.dst)
    ro = oracle.greedy(g.n, g.src, g.dst)
    assert np.array_equal(r["order"].cpu().numpy(), ro["order"])
    assert np.array_equal(r["rem_m"].cpu().numpy(), ro["rem_m"])
    assert (r["num"], r["den"]) == (ro["num"], ro["den"])
    assert np.array_equal(r["in_set"].cpu().numpy(), ro["in_set"])


@pytest.mark.parametrize("name,g", _greedy_graphs()[::5], ids=lambda v: v if isinstance(v, str) else "")
def test_greedy_continues_on_the_pruned_graph(name, g):
    """Theorem 5: greedy on G first removes exactly the nodes Algorithm 2
    removes, and then continues as greedy on the pruned graph H (same
    removal order through the renumbering)."""
    pr = lowd.prune(g.n, g.src, g.dst)
    rg = lowd.greedy_peel(g.n, g.src, g.dst)
    rh = lowd.greedy_peel(pr["n_h"], pr["src"].clone(), pr["dst"].clone())
    order_g = rg["order"].cpu().numpy()
    keep = pr["node_keep"].cpu().numpy()
    k = g.n - pr["n_h"]
    assert set(order_g[:k].tolist()) == set(np.flatnonzero(keep == 0).tolist())
    kept_ids = np.flatnonzero(keep)
    assert np.array_equal(order_g[k:], kept_ids[rh["order"].cpu().numpy()])


def test_prune_then_plugin_solvers():
    """Algorithm 2 with a plug-in DSPSolver on workload 0: LOWD on H reaches
    the max-flow optimum 435/30; greedy on H gives a set of density at least
    half of it (Charikar), both mapped back to G's ids."""
    g = synth.workload(0)
    a = lowd.densest_after_prune(g.n, g.src, g.dst, "lowd", tol=1e-9)
    b = lowd.densest_after_prune(g.n, g.src, g.dst, "greedy")
    assert a["num"] * 30 == 435 * a["den"]
    assert 2 * b["num"] * 30 >= 435 * b["den"]
    for r in (a, b):
        ins = r["in_set"].cpu().numpy().astype(bool)
        assert ins.sum() == r["den"]
        inside = ins[g.src] & ins[g.dst]
        assert inside.sum() == r["num"]


# ------------------------------------------- decomposition read-out --
@pytest.mark.parametrize("T", [0, 3, 40])
@pytest.mark.parametrize("name,g", GRAPHS, ids=[n for n, _ in GRAPHS])
def test_ldd_readout_matches_oracle(name, g, T):
    """The decomposition read from the loads equals the oracle's read-out of
    its own (bit-identical) loads exactly: every level end, f at it (exact
    integer sums, rounded once for weighted graphs) and every node's level."""
    log(f"ldd {name} T={T}")
    sv = lowd.Solver(g.n, g.src, g.dst, g.w, "f64")
    sv.iterate(T)
    r = sv.ldd()
    xo, Lo, *_ = oracle_run(g, T, 16)
    ro = oracle.ldd(g.n, g.src, g.dst, g.w, Lo)
    log(f"  {len(r['k_end'])} levels")
    assert np.array_equal(r["k_end"], ro["k_end"])
    assert np.array_equal(r["f_end"], ro["f_end"])
    assert np.array_equal(r["level"].cpu().numpy(), ro["level"])
    sv.close()


@pytest.mark.parametrize("name,g", GRAPHS[:2], ids=[n for n, _ in GRAPHS[:2]])
def test_convergence_trace_matches_oracle(name, g):
    """lowd_convergence_trace records (sweeps, D, rho, sum of squares, gap)
    every 3 sweeps; each row equals the oracle's state after as many
    sweeps (D exactly, rho exactly for unit weights, sums to 1e-12)."""
    sv = lowd.Solver(g.n, g.src, g.dst, g.w, "f64")
    tr = sv.trace(12, 3)
    assert tr.shape == (5, 5)
    for row in tr:
        T = int(row[0])
        xo, Lo, *_ = oracle_run(g, T, 16)
        ro = oracle.extract(g.n, g.src, g.dst, g.w, Lo)
        Do, _, s2o = oracle.stats(Lo)
        rho = (ro["num"] if g.w is None else ro["num_w"]) / ro["den"]
        assert row[1] == Do
        if g.w is None:
            assert row[2] == rho and row[4] == (Do - rho) / rho
        else:
            assert abs(row[2] - rho) <= 1e-12 * rho
        assert abs(row[3] - s2o) <= 1e-12 * s2o
    sv.close()


def test_ldd_readout_properties_at_full_size():
    """At full size (Chung-Lu 1M nodes / 9.86M edges, 40 sweeps): level 0 is
    the extracted densest set, the level values decrease strictly, the last
    level ends at (n, m), and every level is contiguous in the load order."""
    g = synth.workload(1, seed=1)
    sv = lowd.Solver(g.n, g.src, g.dst, None, "f64")
    sv.iterate(40)
    ex = sv.extract()
    r = sv.ldd()
    ke, fe = r["k_end"], r["f_end"]
    log(f"workload1 ldd: {len(ke)} levels, first {ke[0]} nodes / {fe[0]} edges")
    assert (ke[0], int(fe[0])) == (ex["den"], ex["num"])
    assert ke[-1] == g.n and int(fe[-1]) == g.m
    assert np.all(np.diff(ke) > 0)
    lam = np.diff(np.concatenate([[0.0], fe])) / np.diff(np.concatenate([[0], ke]))
    assert np.all(np.diff(lam) < 0)
    level = r["level"].cpu().numpy()
    assert np.array_equal(level == 0, ex["in_set"].cpu().numpy().astype(bool))
    counts = np.bincount(level, minlength=len(ke))
    assert np.array_equal(np.cumsum(counts), ke)
    sv.close()


# -------------------------------------------------------- batched form --
def batch_graphs(count, seed):
    gs = synth.batch_of_graphs(count, seed=seed, m_lo=20, m_hi=3000)
    rng = np.random.default_rng(seed)
    gs.append(synth.canonical(4, np.zeros(0, np.int64), np.zeros(0, np.int64)))   # no edges
    gs.append(synth.random_small(rng, 9, 0.4))
    gs.append(synth.workload(0))
    return gs


@pytest.mark.parametrize("T", [0, 1, 6])
def test_batch_matches_single_graph_oracle(T):
    """Each graph of the batch equals its own single-graph oracle run:
    loads bit-exact (FP64), densest set and exact density equal."""
    gs = batch_graphs(40, 3)
    log(f"batch of {len(gs)} graphs, T={T}")
    r = lowd.batch_run(gs, T, "f64")
    L = r["load"].cpu().numpy()
    ins = r["in_set"].cpu().numpy()
    for i, g in enumerate(gs):
        a, b = r["node_ptr"][i], r["node_ptr"][i + 1]
        xo, Lo, *_ = oracle_run(g, T, 16)
        assert np.array_equal(L[a:b], Lo), i
        ro = oracle.extract(g.n, g.src, g.dst, None, Lo)
        assert (r["num"][i], r["den"][i]) == (ro["num"], ro["den"]), i
        assert np.array_equal(ins[a:b], ro["in_set"]), i


def test_batch_f32k_within_tolerance():
    gs = batch_graphs(20, 5)
    T = 30
    r = lowd.batch_run(gs, T, "f32k")
    L = r["load"].cpu().numpy()
    for i, g in enumerate(gs):
        a, b = r["node_ptr"][i], r["node_ptr"][i + 1]
        xo, Lo, *_ = oracle_run(g, T, 16)
        if g.m:
            assert np.max(np.abs(L[a:b] - Lo)) <= 1e-5 * np.max(np.abs(Lo)), i


def test_batch_with_several_sort_tiles_per_block():
    """About 275k nodes over 300 graphs: the batched extraction's sorts take
    two tiles per block.  Every graph's densest set and exact density equal
    its own oracle run; after a retire, the next extraction leaves the
    retired graphs' results as they were and gives the others' at 2T."""
    gs = synth.batch_of_graphs(300, seed=29, m_lo=2000, m_hi=6000)
    N = sum(g.n for g in gs)
    log(f"{len(gs)} graphs, N={N}")
    assert N > 1024 * 256
    T, tol = 4, 1e-2
    b = lowd.Batch(gs, "f64")
    b.iterate(T)
    b.extract()
    num, den = b.num.cpu().numpy().copy(), b.den.cpu().numpy().copy()
    ins = b.in_set.cpu().numpy().copy()
    for i, g in enumerate(gs):
        a, c = b.node_ptr[i], b.node_ptr[i + 1]
        _, Lo, *_ = oracle_run(g, T, 16)
        ro = oracle.extract(g.n, g.src, g.dst, None, Lo)
        assert (num[i], den[i]) == (ro["num"], ro["den"]), i
        assert np.array_equal(ins[a:c], ro["in_set"]), i
    retired = b.gaps() <= tol
    active, _ = b.retire(tol)
    log(f"retired {int(retired.sum())}, active {active}")
    assert active == int((~retired).sum()) and 0 < active < len(gs)
    b.iterate(T)
    b.extract()
    num2, den2 = b.num.cpu().numpy(), b.den.cpu().numpy()
    ins2 = b.in_set.cpu().numpy()
    for i, g in enumerate(gs):
        a, c = b.node_ptr[i], b.node_ptr[i + 1]
        if retired[i]:
            assert (num2[i], den2[i]) == (num[i], den[i]), i
            assert np.array_equal(ins2[a:c], ins[a:c]), i
        else:
            _, Lo, *_ = oracle_run(g, 2 * T, 16)
            ro = oracle.extract(g.n, g.src, g.dst, None, Lo)
            assert (num2[i], den2[i]) == (ro["num"], ro["den"]), i
            assert np.array_equal(ins2[a:c], ro["in_set"]), i
    b.close()


def test_prepared_batch_in_steps_equals_oracle():
    """A prepared, autotuned batch run in steps (2 + 3 sweeps) equals the
    oracle's 5 sweeps per graph; D_g is the graph's largest load; a reset
    starts over."""
    gs = batch_graphs(40, 7)
    T = 5
    b = lowd.Batch(gs, "f64", tune=True)
    log(f"prepared batch {b.info()}")
    b.iterate(2)
    b.iterate(3)
    b.extract(loads=True)
    L = b.load.cpu().numpy()
    D = b.D.cpu().numpy()
    num, den = b.num.cpu().numpy(), b.den.cpu().numpy()
    for i, g in enumerate(gs):
        a, c = b.node_ptr[i], b.node_ptr[i + 1]
        xo, Lo, *_ = oracle_run(g, T, 16)
        assert np.array_equal(L[a:c], Lo), i
        assert D[i] == np.max(Lo), i
        ro = oracle.extract(g.n, g.src, g.dst, None, Lo)
        assert (num[i], den[i]) == (ro["num"], ro["den"]), i
    b.reset()
    b.iterate(T)
    b.extract(loads=True)
    assert np.array_equal(b.load.cpu().numpy(), L)
    b.close()


def test_batch_retire_freezes_converged_graphs():
    """After extract + retire(tol), retired graphs keep the oracle's state at
    the retirement sweep while the others continue; the retired set is the
    graphs whose oracle gap is within tol (parity on the set itself)."""
    gs = batch_graphs(40, 13)
    T1, T2, tol = 10, 5, 1e-4
    b = lowd.Batch(gs, "f64")
    b.iterate(T1)
    b.extract()
    num, den, D = b.num.cpu().numpy(), b.den.cpu().numpy(), b.D.cpu().numpy()
    expect_active = []
    for i, g in enumerate(gs):
        xo, Lo, *_ = oracle_run(g, T1, 16)
        ro = oracle.extract(g.n, g.src, g.dst, None, Lo)
        assert (num[i], den[i]) == (ro["num"], ro["den"]) and D[i] == np.max(Lo, initial=0.0), i
        rho = ro["num"] / ro["den"]
        Do = np.max(Lo, initial=0.0)
        gap = (Do - rho) / rho if rho > 0 else (np.inf if Do > 0 else 0.0)
        if gap > tol:
            expect_active.append(i)
    active, active_edges = b.retire(tol)
    log(f"retire: {active} active of {len(gs)}")
    assert active == len(expect_active)
    assert active_edges == sum(gs[i].m for i in expect_active)
    assert 0 < active < len(gs)
    b.iterate(T2)
    b.extract(loads=True)
    L = b.load.cpu().numpy()
    for i, g in enumerate(gs):
        a, c = b.node_ptr[i], b.node_ptr[i + 1]
        T = T1 + T2 if i in expect_active else T1
        xo, Lo, *_ = oracle_run(g, T, 16)
        assert np.array_equal(L[a:c], Lo), i
    b.reset()
    b.iterate(T1 + T2)
    b.extract(loads=True)
    for i, g in enumerate(gs):
        a, c = b.node_ptr[i], b.node_ptr[i + 1]
        xo, Lo, *_ = oracle_run(g, T1 + T2, 16)
        assert np.array_equal(b.load.cpu().numpy()[a:c], Lo), i
    b.close()


@pytest.mark.parametrize("shape", ["8,1,1", "8,0,2", "4,1,2", "4,0,4", "16,0,1"])
def test_batch_every_launch_shape_is_bit_exact(shape, monkeypatch):
    monkeypatch.setenv("LOWD_BATCH_SHAPE", shape)
    gs = batch_graphs(30, 11)
    T = 4
    b = lowd.Batch(gs, "f64")
    info = b.info()
    log(f"shape {shape}: {info}")
    w, pf, pc = (int(v) for v in shape.split(","))
    assert (info["waves"], info["prefetch"]) == (w, pf)
    b.iterate(T)
    b.extract(loads=True)
    L = b.load.cpu().numpy()
    for i, g in enumerate(gs):
        a, c = b.node_ptr[i], b.node_ptr[i + 1]
        xo, Lo, *_ = oracle_run(g, T, 16)
        assert np.array_equal(L[a:c], Lo), i
    b.close()


def test_batch_rejects_bad_graphs():
    g = synth.canonical(5, np.array([0, 1]), np.array([1, 2]))
    bad = synth.Graph(3, np.array([0, 1], np.int32), np.array([1, 5], np.int32), None)
    with pytest.raises(lowd.LowdError) as ei:
        lowd.batch_solve([g, bad])
    assert ei.value.status == -2


def test_batch_f32k_tail_shape_matches_a_fixed_shape(monkeypatch):
    """FP32K batches switch to 16-wave workgroups once few graphs iterate
    (here from the start: 30 graphs); the loads equal, bit for bit, those of
    a forced 8-wave shape, across a retire and further sweeps."""
    gs = batch_graphs(30, 17)
    T1, T2, tol = 6, 4, 1e-3

    def run():
        b = lowd.Batch(gs, "f32k")
        b.iterate(T1)
        b.extract()
        act = b.retire(tol)
        b.iterate(T2)
        b.extract(loads=True)
        out = (b.load.cpu().numpy().copy(), b.num.cpu().numpy().copy(), act)
        b.close()
        return out

    La, na, aa = run()
    monkeypatch.setenv("LOWD_BATCH_SHAPE", "8,1,1")
    Lb, nb, ab = run()
    log(f"active after retire: {aa}")
    assert aa == ab
    assert np.array_equal(La, Lb) and np.array_equal(na, nb)


def test_batch_f32k_bound_is_recomputed_from_the_fractions():
    """FP32K batches report loads (and D_g) recomputed in FP64 from the
    stored FP32 fractions: they match the FP64 sums, on the CPU, of the
    fractions a single-graph FP32K solver holds after the same sweeps (the
    two run the same steps in the same order), and D_g is their maximum."""
    gs = batch_graphs(12, 23)
    T = 20
    b = lowd.Batch(gs, "f32k")
    b.iterate(T)
    b.extract(loads=True)
    L = b.load.cpu().numpy()
    D = b.D.cpu().numpy()
    for i, g in enumerate(gs):
        a, c = b.node_ptr[i], b.node_ptr[i + 1]
        if g.m == 0:
            continue
        sv = lowd.Solver(g.n, g.src, g.dst, None, "f32k")
        sv.iterate(T)
        x, _ = sv.read_state()
        x = x.cpu().numpy()
        ref = np.zeros(g.n)
        np.add.at(ref, g.src, x)
        np.add.at(ref, g.dst, 1.0 - x)
        assert np.max(np.abs(L[a:c] - ref)) <= 1e-12 * np.max(ref), i
        assert D[i] == np.max(L[a:c]), i
        assert abs(D[i] - sv.check()[0]) <= 1e-12 * D[i], i
        sv.close()
    b.close()
