"""Host-side checks of the C interface (no GPU needed): the library loads,
exports every entry point include/lowd.h declares, rejects bad arguments
before touching the device, and its host-built schedule equals the oracle's
schedule definition."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle
import paper_2307_15969_amd as lowd
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "lowd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lowd_[a-z_0-9]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = lowd.lib()
    names = declared_symbols()
    assert len(names) >= 12
    for name in names:
        assert hasattr(L, name), name
    assert lowd.version().startswith("lowd-gfx950")


def test_argument_errors_need_no_device():
    L = lowd.lib()
    h = C.c_void_p()
    # n < 1
    st = L.lowd_init_loads(0, 0, None, None, None, 0, 16, C.byref(h), None)
    assert st == -1 and b"n must be" in L.lowd_last_error()
    assert L.lowd_init_loads(0x7FFFFFFE, 0, None, None, None, 0, 16, C.byref(h), None) == -1
    # bad state / star_max
    assert L.lowd_init_loads(5, 0, None, None, None, 7, 16, C.byref(h), None) == -1
    assert L.lowd_init_loads(5, 0, None, None, None, 0, 0, C.byref(h), None) == -1
    assert L.lowd_init_loads(5, 0, None, None, None, 0, 255, C.byref(h), None) == -1
    # missing arrays
    assert L.lowd_init_loads(5, 3, None, None, None, 0, 16, C.byref(h), None) == -1
    # NULL solver
    assert L.lowd_iterate(None, 1, None) == -1
    assert L.lowd_check(None, None, None, None, None) == -1
    assert L.lowd_check_kept(None, None, None, None, None) == -1
    assert L.lowd_resync_loads(None, None) == -1
    assert L.lowd_extract_densest_kept(None, None, None, None, None, None, None, None) == -1
    assert L.lowd_iterate(None, -1, None) == -1
    L.lowd_solver_free(None)
    assert L.lowd_prune(0, 0, None, None, None, None, None, None, None, None, None, None,
                        None) == -1
    # batches
    b = C.c_void_p()
    assert L.lowd_batch_prepare(0, None, None, None, None, 0, 16, 0, C.byref(b), None) == -1
    ptr = np.array([0, 3], dtype=np.int64)
    zero = np.array([0, 0], dtype=np.int64)
    vp = lambda a: a.ctypes.data_as(C.c_void_p)
    assert L.lowd_batch_prepare(1, vp(ptr), vp(zero), None, None, 0, 16, 2, C.byref(b),
                                None) == -1                               # tune must be 0/1
    assert L.lowd_batch_prepare(1, vp(ptr), vp(zero), None, None, 0, 17, 0, C.byref(b),
                                None) == -1                               # star_max
    assert L.lowd_batch_iterate(None, 1, None) == -1
    assert L.lowd_batch_retire(None, None, None, None, 0.0, None, None, None) == -1
    L.lowd_batch_free(None)


def test_host_schedule_rejects_invalid_edges():
    with pytest.raises(lowd.LowdError) as ei:
        lowd.schedule_build(4, np.array([0, 1]), np.array([1, 1]))
    assert ei.value.status == -2
    with pytest.raises(lowd.LowdError):
        lowd.schedule_build(4, np.array([0, 5]), np.array([1, 2]))


@pytest.mark.parametrize("smax", [1, 2, 5, 16, 32, 64])
def test_host_schedule_equals_oracle_schedule(smax):
    graphs = [synth.workload(0)]
    rng = np.random.default_rng(smax)
    for _ in range(4):
        graphs.append(synth.random_small(rng, int(rng.integers(5, 300)), float(rng.uniform(0.01, 0.5))))
    graphs.append(synth.chung_lu(20000, 200000, 2.1, seed=3, planted=50, p_planted=0.3))
    for g in graphs:
        p1, c1, P1 = lowd.schedule_build(g.n, g.src, g.dst, smax)
        p2, c2, _, P2 = oracle.schedule(g.n, g.src, g.dst, smax)
        assert P1 == P2
        assert np.array_equal(p1, p2)
        assert np.array_equal(c1, c2)


def test_host_schedule_empty_graph():
    p, c, P = lowd.schedule_build(3, np.zeros(0, np.int32), np.zeros(0, np.int32))
    assert P == 0 and p.size == 0


def test_dks_bound_host_function_equals_oracle():
    """lowd_dks_bound (host only) evaluates Corollary 1's envelope like the
    oracle's helper, on random decompositions; argument errors are caught."""
    rng = np.random.default_rng(3)
    for _ in range(50):
        L = int(rng.integers(1, 8))
        ke = np.cumsum(rng.integers(1, 20, size=L)).astype(np.int64)
        slopes = np.sort(rng.uniform(0.1, 10.0, size=L))[::-1]
        fe = np.cumsum(slopes * np.diff(np.concatenate([[0], ke])))
        for k in range(1, int(ke[-1]) + 1):
            assert abs(lowd.dks_bound(ke, fe, k) - oracle.dks_bound(ke, fe, k)) <= 1e-12
    with pytest.raises(lowd.LowdError):
        lowd.dks_bound(np.array([3], np.int64), np.array([2.0]), 4)
