"""lowd_prune_noalloc against lowd_prune, through the C interface.

The allocation-free prune takes every device buffer from the library's fixed
scratch array; its results must equal the allocating prune's bit for bit, on
two calls in a row, the second with a smaller graph (the scratch keeps the
first call's contents, so anything the call does not clear would show up).
A graph whose buffers exceed the scratch is rejected on the host.
"""
import ctypes as C

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2307_15969_amd as lowd  # noqa: E402


def _same(a, b):
    assert (a["rounds"], a["n_h"], a["m_h"]) == (b["rounds"], b["n_h"], b["m_h"])
    for k in ("node_keep", "relabel", "src", "dst", "edge_map"):
        assert torch.equal(a[k], b[k]), k


def test_noalloc_prune_equals_prune_on_two_calls():
    big = synth.rmat(16, 16, seed=4)        # ~0.9M edges
    small = synth.rmat(12, 16, seed=5)      # the second call: a smaller graph
    for g in (big, small):
        print(f"prune_noalloc: n={g.n} m={g.m}", flush=True)
        src = torch.from_numpy(g.src).cuda()
        dst = torch.from_numpy(g.dst).cuda()
        ref = lowd.prune(g.n, src, dst)
        got = lowd.prune(g.n, src, dst, noalloc=True)
        torch.cuda.synchronize()
        _same(got, ref)
        assert 0 < got["n_h"] < g.n


def test_noalloc_prune_rejects_a_graph_beyond_its_scratch():
    # the size check runs on the host before any device work; the arrays are
    # never read
    src = torch.zeros(1, dtype=torch.int32, device="cuda")
    keep = torch.zeros(1, dtype=torch.uint8, device="cuda")
    r, nh, mh = C.c_int32(), C.c_int32(), C.c_int64()
    st = lowd.lib().lowd_prune_noalloc(1 << 24, 1 << 28, C.c_void_p(src.data_ptr()),
                                       C.c_void_p(src.data_ptr()), C.c_void_p(keep.data_ptr()),
                                       None, None, None, None, C.byref(r), C.byref(nh),
                                       C.byref(mh), None)
    assert st == -5
    assert b"bytes of scratch" in lowd.lib().lowd_last_error()
