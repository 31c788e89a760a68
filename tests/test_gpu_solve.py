"""GPU parity of the solves to a tolerance and of the workloads' own shapes.

- lowd_solve (Section III-B's stopping rule behind the C interface): the
  bound D it returns equals the oracle's largest load after as many sweeps
  (bit for bit in FP64), the returned set is a set of the graph with the
  stated exact density, and the certified gap holds with the oracle's D.
- lowd_batch_solve (one persistent launch; every graph checked and stopped
  inside its workgroup) on a batch shaped like the 4096-graph workload (edge
  targets log-uniform up to 50,000, planted blocks), both states: every
  graph's set and exact density equal the FP64 oracle's extraction after the
  sweeps the set was taken at, and its D the oracle's largest load after all
  of the graph's sweeps (bit for bit in FP64, within 1e-5 in FP32K).
- The pruned graph of an R-MAT graph (the shape of the scale-24 workload: a
  hub adjacent to nearly every node, hundreds of phases, the LDS tier):
  FP64 bit-exact on every tier split, FP32K within 1e-5, the same set.
- Edge lists in arbitrary order and orientation.
"""
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


def oracle_state(g, T, src=None, dst=None, w=None, smax=16):
    """oracle schedule, init and T sweeps on (src, dst, w) (default: g's)"""
    s = g.src if src is None else src
    d = g.dst if dst is None else dst
    ww = g.w if src is None else w
    phase, center, order, P = oracle.schedule(g.n, s, d, smax)
    x, L = oracle.init(g.n, s, d, ww)
    oracle.sweep(g.n, s, d, ww, order, T, x, L)
    return x, L, phase


def induced(src, dst, w, in_set):
    """(edges, weight) of the subgraph induced by in_set"""
    k = in_set[src].astype(bool) & in_set[dst].astype(bool)
    return int(k.sum()), (float(w[k].astype(np.float64).sum()) if w is not None else None)


TOL = 1e-6


# ------------------------------------------------------------- lowd_solve --
SOLVE_GRAPHS = [("workload0", synth.workload(0)),
                ("chunglu20k", synth.chung_lu(20000, 200000, 2.1, seed=3, planted=60,
                                              p_planted=0.3)),
                ("chunglu15k_w", synth.chung_lu(15000, 120000, 2.1, seed=4,
                                                weights="lognormal"))]


@pytest.mark.parametrize("name,g", SOLVE_GRAPHS, ids=[n for n, _ in SOLVE_GRAPHS])
def test_solve_f64_certifies_with_the_oracle_bound(name, g):
    sv = lowd.Solver(g.n, g.src, g.dst, g.w, "f64")
    r = sv.solve(TOL)
    assert r["converged"]
    T = r["sweeps"]
    x, L = sv.read_state()
    xo, Lo, _ = oracle_state(g, T)
    assert np.array_equal(L.cpu().numpy(), Lo) and np.array_equal(x.cpu().numpy(), xo)
    # the returned D is the oracle's largest load after the same sweeps
    assert r["D"] == float(Lo.max())
    ins = r["in_set"].cpu().numpy()
    e, wsum = induced(g.src, g.dst, g.w, ins)
    assert int(ins.sum()) == r["den"]
    if g.w is None:
        assert e == r["num"]
        rho = r["num"] / r["den"]
    else:
        assert abs(wsum - r["num_w"]) <= 1e-12 * wsum
        rho = r["num_w"] / r["den"]
    assert (Lo.max() - rho) / rho <= TOL
    # the returned set is at least as dense as the oracle's extraction at the end
    ro = oracle.extract(g.n, g.src, g.dst, g.w, Lo)
    rho_o = (ro["num"] if g.w is None else ro["num_w"]) / ro["den"]
    assert rho >= rho_o * (1 - 1e-15)
    if name == "workload0":
        assert (r["num"], r["den"]) == (435, 30)
    log(f"  {name}: {T} sweeps, gap {r['gap']:.2e}, density {rho}")
    sv.close()


@pytest.mark.parametrize("name,g", SOLVE_GRAPHS, ids=[n for n, _ in SOLVE_GRAPHS])
def test_solve_f32k_bound_is_the_fractions_bound(name, g):
    """FP32K: the certified D is that of the stored fractions (lowd_check
    recomputes it), within the tolerance; loads within 1e-5 of the FP64
    oracle after the same sweeps; the set's density within the tolerance
    of the FP64 solve's."""
    sv = lowd.Solver(g.n, g.src, g.dst, g.w, "f32k")
    r = sv.solve(TOL)
    assert r["converged"]
    assert r["D"] == sv.check()[0]
    rho = (r["num"] if g.w is None else r["num_w"]) / r["den"]
    assert (r["D"] - rho) / rho <= TOL
    _, L = sv.read_state()
    _, Lo, _ = oracle_state(g, r["sweeps"])
    assert np.max(np.abs(L.cpu().numpy() - Lo)) <= 1e-5 * np.max(np.abs(Lo))
    r64 = lowd.solve(g.n, g.src, g.dst, g.w, "f64", tol=TOL)
    rho64 = (r64["num"] if g.w is None else r64["num_w"]) / r64["den"]
    assert abs(rho - rho64) <= 2 * TOL * rho64
    log(f"  {name}: f32k {r['sweeps']} sweeps, f64 {r64['sweeps']}")
    sv.close()


def test_solve_reports_not_converged():
    g = SOLVE_GRAPHS[1][1]
    sv = lowd.Solver(g.n, g.src, g.dst, None, "f64")
    r = sv.solve(1e-14, max_sweeps=3, check_every=2)
    assert not r["converged"] and r["sweeps"] == 3 and r["gap"] > 1e-14
    _, Lo, _ = oracle_state(g, 3)
    assert r["D"] == float(Lo.max())
    # continuing from the state reached: the remaining sweeps to the tolerance
    r2 = sv.solve(TOL)
    assert r2["converged"]
    sv.reset()
    r3 = sv.solve(TOL)
    assert r3["converged"] and r3["sweeps"] >= r2["sweeps"]
    sv.close()


# ---------------------------------------------------- input order -------
def _shuffled(g, seed):
    rng = np.random.default_rng(seed)
    perm = rng.permutation(g.m)
    flip = rng.random(g.m) < 0.5
    s = np.ascontiguousarray(np.where(flip, g.dst, g.src)[perm], dtype=np.int32)
    d = np.ascontiguousarray(np.where(flip, g.src, g.dst)[perm], dtype=np.int32)
    w = None if g.w is None else np.ascontiguousarray(g.w[perm])
    return s, d, w


@pytest.mark.parametrize("name,g", SOLVE_GRAPHS, ids=[n for n, _ in SOLVE_GRAPHS])
def test_shuffled_mixed_orientation_edge_list(name, g):
    """An edge list in random order, each edge in random orientation: the
    schedule, fractions, loads and extraction equal the oracle's on the same
    arrays, bit for bit (FP64)."""
    s, d, w = _shuffled(g, 11)
    T = 5
    sv = lowd.Solver(g.n, s, d, w, "f64")
    sv.iterate(T)
    x, L = sv.read_state()
    xo, Lo, phase_o = oracle_state(g, T, s, d, w)
    phase, _, _ = sv.schedule()
    assert np.array_equal(phase, phase_o)
    assert np.array_equal(x.cpu().numpy(), xo)
    assert np.array_equal(L.cpu().numpy(), Lo)
    ex = sv.extract()
    ro = oracle.extract(g.n, s, d, w, Lo)
    assert np.array_equal(ex["in_set"].cpu().numpy(), ro["in_set"])
    assert ex["den"] == ro["den"]
    if w is None:
        assert ex["num"] == ro["num"]
    sv.close()


def test_shuffled_edge_list_prune():
    g = synth.rmat(14, 16, seed=2)
    s, d, _ = _shuffled(g, 12)
    pr = lowd.prune(g.n, s, d)
    keep, rounds, nh, mh = oracle.prune(g.n, s, d)
    assert np.array_equal(pr["node_keep"].cpu().numpy(), keep)
    assert (pr["rounds"], pr["n_h"], pr["m_h"]) == (rounds, nh, mh)
    # H's edges: the kept edges in their input order, in H's ids
    relabel = np.cumsum(keep) - 1
    k = keep[s].astype(bool) & keep[d].astype(bool)
    assert np.array_equal(pr["src"].cpu().numpy(), relabel[s[k]])
    assert np.array_equal(pr["dst"].cpu().numpy(), relabel[d[k]])


# ------------------------------------------- the pruned R-MAT graph ------
@pytest.fixture(scope="module")
def rmat_h():
    g = synth.rmat(19, 16, seed=3)
    keep, rounds, nh, mh = oracle.prune(g.n, g.src, g.dst)
    relabel = np.cumsum(keep) - 1
    k = keep[g.src].astype(bool) & keep[g.dst].astype(bool)
    h = synth.Graph(int(nh), relabel[g.src[k]].astype(np.int32),
                    relabel[g.dst[k]].astype(np.int32), None, "rmat19_H")
    log(f"rmat19: {g.m} edges -> H {h.n} nodes, {h.m} edges, {rounds} rounds")
    return g, h


SPLITS = {"auto": (None, None), "all_lds": (0, None), "no_lds": (1 << 30, 1 << 30),
          "all_mid": (1 << 30, 0), "mid_lds": (None, 0)}


@pytest.mark.parametrize("smax", [16, 32])
@pytest.mark.parametrize("tier", list(SPLITS))
def test_pruned_rmat_h_sweeps_bit_exact(rmat_h, tier, smax, monkeypatch):
    g, h = rmat_h
    tail, mid = SPLITS[tier]
    for var, v in (("LOWD_TAIL_SPLIT", tail), ("LOWD_MID_SPLIT", mid)):
        if v is None:
            monkeypatch.delenv(var, raising=False)
        else:
            monkeypatch.setenv(var, str(v))
    pr = lowd.prune(g.n, g.src, g.dst)
    assert pr["n_h"] == h.n and pr["m_h"] == h.m
    assert np.array_equal(pr["src"].cpu().numpy(), h.src)
    assert np.array_equal(pr["dst"].cpu().numpy(), h.dst)
    T = 3
    sv = lowd.Solver(h.n, pr["src"].clone(), pr["dst"].clone(), None, "f64", star_max=smax)
    info = sv.info()
    log(f"  {tier} smax={smax}: {info}")
    sv.iterate(T)
    x, L = sv.read_state()
    xo, Lo, _ = oracle_state(h, T, smax=smax)
    assert np.array_equal(x.cpu().numpy(), xo)
    assert np.array_equal(L.cpu().numpy(), Lo)
    ex = sv.extract()
    ro = oracle.extract(h.n, h.src, h.dst, None, Lo)
    assert (ex["num"], ex["den"]) == (ro["num"], ro["den"])
    assert np.array_equal(ex["in_set"].cpu().numpy(), ro["in_set"])
    sv.close()


@pytest.mark.parametrize("smax", [16, 32])
def test_pruned_rmat_h_f32k_and_solve(rmat_h, smax):
    """FP32K on H within 1e-5 of the FP64 oracle; both states solved to the
    tolerance give the same densest set, and the FP64 one equals the
    oracle's extraction after its sweeps."""
    _, h = rmat_h
    T = 6
    sv = lowd.Solver(h.n, h.src, h.dst, None, "f32k", star_max=smax)
    sv.iterate(T)
    _, L = sv.read_state()
    _, Lo, _ = oracle_state(h, T, smax=smax)
    assert np.max(np.abs(L.cpu().numpy() - Lo)) <= 1e-5 * np.max(np.abs(Lo))
    sv.reset()
    r32 = sv.solve(TOL)
    sv.close()
    sv = lowd.Solver(h.n, h.src, h.dst, None, "f64", star_max=smax)
    r64 = sv.solve(TOL)
    sv.close()
    assert r32["converged"] and r64["converged"]
    _, Lo, _ = oracle_state(h, r64["sweeps"], smax=smax)
    ro = oracle.extract(h.n, h.src, h.dst, None, Lo)
    assert r64["D"] == float(Lo.max())
    assert (r64["num"], r64["den"]) == (ro["num"], ro["den"])
    assert (r32["num"], r32["den"]) == (r64["num"], r64["den"])
    assert np.array_equal(r32["in_set"].cpu().numpy(), r64["in_set"].cpu().numpy())
    log(f"  H: f64 {r64['sweeps']} sweeps, f32k {r32['sweeps']}, density "
        f"{r64['num']}/{r64['den']}")


# ------------------------------------------ the batch, at its own shape --
def config5_batch():
    """Graphs drawn like the 4096-graph workload (edge targets log-uniform in
    [100, 50000]), plus two graphs above 40,000 edges (the largest LDS
    budget), a graph without edges and the 1000-node correctness graph."""
    gs = synth.batch_of_graphs(60, seed=7)
    gs += synth.batch_of_graphs(2, seed=8, m_lo=40000, m_hi=50000)
    gs.append(synth.canonical(6, np.zeros(0, np.int64), np.zeros(0, np.int64)))
    gs.append(synth.workload(0))
    return gs


@pytest.mark.parametrize("state", ["f64", "f32k"])
def test_batch_solve_at_the_workload_shape(state):
    gs = config5_batch()
    assert sum(g.m > 40000 for g in gs) >= 2
    b = lowd.Batch(gs, state)
    info = b.info()
    log(f"  {state}: {info}")
    assert info["lds"] > 64 * 1024
    r = b.solve(TOL)
    assert r["converged"]
    num, den, D = b.num.cpu().numpy(), b.den.cpu().numpy(), b.D.cpu().numpy()
    ins = b.in_set.cpu().numpy()
    for i, g in enumerate(gs):
        a, c = b.node_ptr[i], b.node_ptr[i + 1]
        T, Ts = int(r["sweeps"][i]), int(r["set_sweeps"][i])
        assert 0 < Ts <= T
        # the set: the oracle's extraction after the sweeps it was taken at
        _, Ls, _ = oracle_state(g, Ts)
        ro = oracle.extract(g.n, g.src, g.dst, None, Ls)
        assert (num[i], den[i]) == (ro["num"], ro["den"]), (i, g.m, Ts)
        assert np.array_equal(ins[a:c], ro["in_set"]), (i, g.m, Ts)
        if g.m == 0:
            continue
        # the bound: the oracle's largest load after all the graph's sweeps
        _, Lo, _ = oracle_state(g, T)
        Do = float(Lo.max())
        if state == "f64":
            assert D[i] == Do, i
        else:
            assert abs(D[i] - Do) <= 1e-5 * Do, i
        rho = num[i] / den[i]
        assert (D[i] - rho) / rho <= TOL, i
    log(f"  {state}: sweeps {int(r['sweeps'].min())}..{int(r['sweeps'].max())}")
    b.reset()
    r2 = b.solve(TOL)
    assert np.array_equal(r2["sweeps"], r["sweeps"])
    assert np.array_equal(b.num.cpu().numpy(), num)
    assert np.array_equal(b.in_set.cpu().numpy(), ins)
    b.close()


@pytest.mark.parametrize("shape", ["4,0,2", "4,1,1", "8,0,1"])
def test_batch_solve_every_launch_shape_agrees(shape, monkeypatch):
    """The launch shape changes only which workgroup runs which graph: the
    sweep counts and sets are the same for every shape."""
    gs = synth.batch_of_graphs(40, seed=21, m_lo=100, m_hi=8000)
    ref = lowd.batch_solve(gs, TOL, "f64")
    monkeypatch.setenv("LOWD_BATCH_SHAPE", shape)
    r = lowd.batch_solve(gs, TOL, "f64")
    assert np.array_equal(r["sweeps"], ref["sweeps"])
    assert np.array_equal(r["set_sweeps"], ref["set_sweeps"])
    assert np.array_equal(r["num"], ref["num"]) and np.array_equal(r["den"], ref["den"])
    assert np.array_equal(r["in_set"].cpu().numpy(), ref["in_set"].cpu().numpy())
    assert np.array_equal(r["D"], ref["D"])


def test_batch_solve_reports_not_converged():
    gs = synth.batch_of_graphs(12, seed=9, m_lo=200, m_hi=2000)
    r = lowd.batch_solve(gs, 1e-14, "f64", max_sweeps=4, check_every=2)
    assert not r["converged"]
    assert int(r["sweeps"].max()) == 4


# ------------------------------------------- node-indexed load layout ----
NODE_GRAPHS = SOLVE_GRAPHS + [("uniform_2^13_2^17", synth.uniform_pairs(13, 17, seed=3))]


@pytest.mark.parametrize("smax", [1, 16, 32])
@pytest.mark.parametrize("name,g", NODE_GRAPHS, ids=[n for n, _ in NODE_GRAPHS])
def test_node_layout_sweeps_bit_exact(name, g, smax, monkeypatch):
    """Loads in a node-indexed array (the layout for wide phases): the same
    bits as the oracle's sequential loop, across launches with eager work in
    between; D, the extraction and the initial state after a reset too."""
    monkeypatch.setenv("LOWD_LAYOUT", "node")
    sv = lowd.Solver(g.n, g.src, g.dst, g.w, "f64", star_max=smax)
    info = sv.info()
    assert info["node_layout"] == 1 and info["lds_phases"] == 0 and info["mid_phases"] == 0
    T = 7
    sv.iterate(1)
    sv.check()
    sv.iterate(2)
    sv.extract()
    sv.iterate(T - 3)
    x, L = sv.read_state()
    xo, Lo, _ = oracle_state(g, T, smax=smax)
    assert np.array_equal(x.cpu().numpy(), xo)
    assert np.array_equal(L.cpu().numpy(), Lo)
    assert sv.check()[0] == float(Lo.max())
    ex = sv.extract()
    ro = oracle.extract(g.n, g.src, g.dst, g.w, Lo)
    assert np.array_equal(ex["in_set"].cpu().numpy(), ro["in_set"])
    assert ex["den"] == ro["den"] and ex["num_w"] == ro["num_w"]
    sv.reset()
    x0, L0 = sv.read_state()
    xi, Li = oracle.init(g.n, g.src, g.dst, g.w)
    assert np.array_equal(x0.cpu().numpy(), xi) and np.array_equal(L0.cpu().numpy(), Li)
    sv.close()


@pytest.mark.parametrize("name,g", NODE_GRAPHS, ids=[n for n, _ in NODE_GRAPHS])
def test_node_layout_f32k_and_solve(name, g, monkeypatch):
    monkeypatch.setenv("LOWD_LAYOUT", "node")
    sv = lowd.Solver(g.n, g.src, g.dst, g.w, "f32k")
    assert sv.info()["node_layout"] == 1
    sv.iterate(6)
    _, L = sv.read_state()
    _, Lo, _ = oracle_state(g, 6)
    assert np.max(np.abs(L.cpu().numpy() - Lo)) <= 1e-5 * np.max(np.abs(Lo))
    sv.reset()
    r = sv.solve(TOL)
    assert r["converged"] and r["D"] == sv.check()[0]
    sv.close()
    sv = lowd.Solver(g.n, g.src, g.dst, g.w, "f64")
    r64 = sv.solve(TOL)
    _, Lo, _ = oracle_state(g, r64["sweeps"])
    assert r64["D"] == float(Lo.max())
    sv.close()


# ------------------------------------------------------- pulled phases ----
# Whole-GPU phases of at least LOWD_PULL_EDGES edges gather each node's load
# from its previous station (which keeps its output) instead of receiving it
# at their own; 0 pulls every whole-GPU phase, the other thresholds mix
# pulled and pushed phases, so every transition (push to pull, pull to
# push, pull to pull, and the wrap into the next sweep) occurs.
PULL_GRAPHS = NODE_GRAPHS


@pytest.mark.parametrize("tier", ["auto", "no_lds", "all_mid"])
@pytest.mark.parametrize("pull_edges", [0, 300, 3000])
@pytest.mark.parametrize("smax", [16, 32])
@pytest.mark.parametrize("name,g", PULL_GRAPHS, ids=[n for n, _ in PULL_GRAPHS])
def test_pulled_phases_sweep_bit_exact(name, g, smax, pull_edges, tier, monkeypatch):
    """The same bits as the oracle's sequential loop with pulled whole-GPU
    phases, across launches with eager work in between; D, the extraction,
    and the initial state after a reset (each node's load where its first
    station reads it) too."""
    monkeypatch.setenv("LOWD_PULL_EDGES", str(pull_edges))
    tail, mid = {"auto": (None, None), "no_lds": (1 << 30, 1 << 30), "all_mid": (1 << 30, 0)}[tier]
    for var, v in (("LOWD_TAIL_SPLIT", tail), ("LOWD_MID_SPLIT", mid)):
        if v is None:
            monkeypatch.delenv(var, raising=False)
        else:
            monkeypatch.setenv(var, str(v))
    sv = lowd.Solver(g.n, g.src, g.dst, g.w, "f64", star_max=smax)
    info = sv.info()
    log(f"pull {name} smax={smax} edges>={pull_edges} tier={tier}: {info}")
    if pull_edges == 0:
        assert info["pulled_phases"] == info["grid_phases"]
    T = 7
    sv.iterate(1)
    sv.check()
    sv.iterate(2)
    sv.extract()
    sv.iterate(T - 3)
    x, L = sv.read_state()
    xo, Lo, _ = oracle_state(g, T, smax=smax)
    assert np.array_equal(L.cpu().numpy(), Lo), np.flatnonzero(L.cpu().numpy() != Lo)[:10]
    assert np.array_equal(x.cpu().numpy(), xo)
    assert sv.check()[0] == float(Lo.max())
    ex = sv.extract()
    ro = oracle.extract(g.n, g.src, g.dst, g.w, Lo)
    assert np.array_equal(ex["in_set"].cpu().numpy(), ro["in_set"])
    assert ex["den"] == ro["den"] and ex["num_w"] == ro["num_w"]
    sv.reset()
    x0, L0 = sv.read_state()
    xi, Li = oracle.init(g.n, g.src, g.dst, g.w)
    assert np.array_equal(x0.cpu().numpy(), xi) and np.array_equal(L0.cpu().numpy(), Li)
    sv.iterate(2)
    x2, L2 = sv.read_state()
    xo2, Lo2, _ = oracle_state(g, 2, smax=smax)
    assert np.array_equal(L2.cpu().numpy(), Lo2) and np.array_equal(x2.cpu().numpy(), xo2)
    sv.close()


@pytest.mark.parametrize("pull_edges", [0, 300])
@pytest.mark.parametrize("name,g", PULL_GRAPHS, ids=[n for n, _ in PULL_GRAPHS])
def test_pulled_phases_f32k_and_solve(name, g, pull_edges, monkeypatch):
    """FP32K with pulled phases within 1e-5 of the FP64 oracle; the kept-load
    screen, the resync from the fractions and the solve find the bound the
    state's loads give; the FP64 solve's D is the oracle's."""
    monkeypatch.setenv("LOWD_PULL_EDGES", str(pull_edges))
    sv = lowd.Solver(g.n, g.src, g.dst, g.w, "f32k")
    info = sv.info()
    if pull_edges == 0:
        assert info["pulled_phases"] == info["grid_phases"]
    sv.iterate(6)
    _, L = sv.read_state()
    _, Lo, _ = oracle_state(g, 6)
    assert np.max(np.abs(L.cpu().numpy() - Lo)) <= 1e-5 * np.max(np.abs(Lo))
    sv.reset()
    r = sv.solve(TOL)
    assert r["converged"] and r["D"] == sv.check()[0]
    sv.close()
    sv = lowd.Solver(g.n, g.src, g.dst, g.w, "f64")
    r64 = sv.solve(TOL)
    _, Lo, _ = oracle_state(g, r64["sweeps"])
    assert r64["D"] == float(Lo.max())
    sv.close()
