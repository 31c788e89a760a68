"""Python binding of liblowd.so, the gfx950 implementation of LOWD (Locally
Optimal Weight Distribution, Algorithm 1) and its pruning pre-process
(Algorithm 2) from arXiv 2307.15969.

The binding only marshals arguments: PyTorch supplies device memory and the
current HIP stream; every step runs in the library's HIP kernels.  There is
no CPU fallback: if the library is missing, every call raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblowd.so")

LOWD_OK = 0
STATE_F64 = 0
STATE_F32K = 1
_STATES = {"f64": STATE_F64, "f32k": STATE_F32K}

_lib = None


class LowdError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"lowd status {status}: {msg}")
        self.status = status


def lib() -> C.CDLL:
    """The loaded liblowd.so (built by paper_2307_15969_amd.build)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LowdError(-5, f"{LIB_PATH} is missing: run paper_2307_15969_amd/build.py")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64 = C.c_void_p, C.c_int32, C.c_int64
        P = C.POINTER
        L.lowd_version.restype = C.c_char_p
        L.lowd_last_error.restype = C.c_char_p
        L.lowd_prune.argtypes = [i32, i64, vp, vp, vp, vp, vp, vp, vp, P(i32), P(i32), P(i64), vp]
        L.lowd_prune_noalloc.argtypes = L.lowd_prune.argtypes
        L.lowd_prune_weighted.argtypes = [i32, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, P(i32),
                                          P(i32), P(i64), P(C.c_double), vp]
        L.lowd_greedy_peel.argtypes = [i32, i64, vp, vp, vp, vp, vp, P(i64), P(i64), vp]
        L.lowd_init_loads.argtypes = [i32, i64, vp, vp, vp, i32, i32, P(vp), vp]
        L.lowd_iterate.argtypes = [vp, i32, vp]
        L.lowd_reset_loads.argtypes = [vp, vp]
        L.lowd_check.argtypes = [vp, P(C.c_double), P(C.c_double), P(C.c_double), vp]
        L.lowd_extract_densest.argtypes = [vp, vp, P(i64), P(C.c_double), P(i64),
                                           P(C.c_double), P(C.c_double), vp]
        L.lowd_check_kept.argtypes = L.lowd_check.argtypes
        L.lowd_solve.argtypes = [vp, C.c_double, i32, i32, vp, P(i64), P(C.c_double), P(i64),
                                 P(C.c_double), P(C.c_double), P(i32), vp]
        L.lowd_resync_loads.argtypes = [vp, vp]
        L.lowd_extract_densest_kept.argtypes = L.lowd_extract_densest.argtypes
        L.lowd_read_state.argtypes = [vp, vp, vp, vp]
        L.lowd_ldd_readout.argtypes = [vp, vp, vp, vp, P(i64), vp]
        L.lowd_convergence_trace.argtypes = [vp, i32, i32, vp, P(i64), vp]
        L.lowd_dks_bound.argtypes = [vp, vp, i64, i64, P(C.c_double)]
        L.lowd_schedule_export.argtypes = [vp, vp, vp, P(i32)]
        L.lowd_solver_info.argtypes = [vp, vp]
        L.lowd_schedule_build.argtypes = [i32, i64, vp, vp, i32, vp, vp, P(i32)]
        L.lowd_solver_free.argtypes = [vp]
        L.lowd_solver_free.restype = None
        L.lowd_batch_solve.argtypes = [i32, vp, vp, vp, vp, i32, i32, C.c_double, i32, i32, vp, vp,
                                       vp, vp, vp, vp, vp]
        L.lowd_batch_solve_prepared.argtypes = [vp, C.c_double, i32, i32, vp, vp, vp, vp, vp, vp,
                                                vp]
        L.lowd_batch_prepare.argtypes = [i32, vp, vp, vp, vp, i32, i32, i32, P(vp), vp]
        L.lowd_batch_reset.argtypes = [vp, vp]
        L.lowd_batch_iterate.argtypes = [vp, i32, vp]
        L.lowd_batch_extract.argtypes = [vp, vp, vp, vp, vp, vp, vp]
        L.lowd_batch_info.argtypes = [vp, vp]
        L.lowd_batch_retire.argtypes = [vp, vp, vp, vp, C.c_double, P(i32), P(i64), vp]
        L.lowd_batch_free.argtypes = [vp]
        L.lowd_batch_free.restype = None
        for f in (L.lowd_prune, L.lowd_prune_noalloc, L.lowd_prune_weighted, L.lowd_greedy_peel, L.lowd_init_loads, L.lowd_iterate, L.lowd_check,
                  L.lowd_extract_densest, L.lowd_read_state, L.lowd_schedule_export,
                  L.lowd_ldd_readout, L.lowd_convergence_trace, L.lowd_dks_bound,
                  L.lowd_solver_info, L.lowd_batch_solve, L.lowd_schedule_build, L.lowd_reset_loads,
                  L.lowd_batch_prepare, L.lowd_batch_reset, L.lowd_batch_iterate,
                  L.lowd_batch_extract, L.lowd_batch_info, L.lowd_batch_retire,
                  L.lowd_check_kept, L.lowd_extract_densest_kept, L.lowd_resync_loads,
                  L.lowd_solve, L.lowd_batch_solve_prepared):
            f.restype = C.c_int32
        _lib = L
    return _lib


def _check(status: int):
    if status < 0:
        raise LowdError(status, lib().lowd_last_error().decode())
    return status


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _dev(t, dtype, name, allow_none=False):
    torch = _torch()
    if t is None:
        if allow_none:
            return None
        raise ValueError(f"{name} is required")
    if not isinstance(t, torch.Tensor):
        t = torch.as_tensor(np.ascontiguousarray(t))
    if t.dtype != dtype:
        t = t.to(dtype)
    if not t.is_cuda:
        t = t.cuda()
    return t.contiguous()


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def prune(n: int, src, dst, stream=None, noalloc: bool = False) -> dict:
    """Algorithm 2 on an unweighted graph (device arrays) -> dict with the
    node mask, the renumbering, the compacted edge list of H and its sizes.
    noalloc: lowd_prune_noalloc (the library's fixed scratch, no device
    allocation inside the call)."""
    torch = _torch()
    s = _dev(src, torch.int32, "src")
    d = _dev(dst, torch.int32, "dst")
    m = s.numel()
    keep = torch.empty(n, dtype=torch.uint8, device=s.device)
    relabel = torch.empty(n, dtype=torch.int32, device=s.device)
    hs = torch.empty(max(m, 1), dtype=torch.int32, device=s.device)
    hd = torch.empty(max(m, 1), dtype=torch.int32, device=s.device)
    emap = torch.empty(max(m, 1), dtype=torch.int64, device=s.device)
    r, nh, mh = C.c_int32(0), C.c_int32(0), C.c_int64(0)
    f = lib().lowd_prune_noalloc if noalloc else lib().lowd_prune
    _check(f(n, m, _ptr(s), _ptr(d), _ptr(keep), _ptr(relabel), _ptr(hs), _ptr(hd), _ptr(emap),
             C.byref(r), C.byref(nh), C.byref(mh), _stream(stream)))
    mh = int(mh.value)
    return dict(node_keep=keep, relabel=relabel, src=hs[:mh], dst=hd[:mh], edge_map=emap[:mh],
                rounds=int(r.value), n_h=int(nh.value), m_h=mh)


def prune_weighted(n: int, src, dst, w, stream=None) -> dict:
    """Algorithm 2 on a weighted graph, decided exactly (lowd_prune_weighted):
    like prune(), plus H's edge weights and its total weight w_h."""
    torch = _torch()
    s = _dev(src, torch.int32, "src")
    d = _dev(dst, torch.int32, "dst")
    ww = _dev(w, torch.float32, "w")
    m = s.numel()
    keep = torch.empty(n, dtype=torch.uint8, device=s.device)
    relabel = torch.empty(n, dtype=torch.int32, device=s.device)
    hs = torch.empty(max(m, 1), dtype=torch.int32, device=s.device)
    hd = torch.empty(max(m, 1), dtype=torch.int32, device=s.device)
    hw = torch.empty(max(m, 1), dtype=torch.float32, device=s.device)
    emap = torch.empty(max(m, 1), dtype=torch.int64, device=s.device)
    r, nh, mh, wh = C.c_int32(0), C.c_int32(0), C.c_int64(0), C.c_double(0)
    _check(lib().lowd_prune_weighted(n, m, _ptr(s), _ptr(d), _ptr(ww), _ptr(keep), _ptr(relabel),
                                     _ptr(hs), _ptr(hd), _ptr(hw), _ptr(emap), C.byref(r),
                                     C.byref(nh), C.byref(mh), C.byref(wh), _stream(stream)))
    mh = int(mh.value)
    return dict(node_keep=keep, relabel=relabel, src=hs[:mh], dst=hd[:mh], w=hw[:mh],
                edge_map=emap[:mh], rounds=int(r.value), n_h=int(nh.value), m_h=mh,
                w_h=float(wh.value))


def greedy_peel(n: int, src, dst, stream=None) -> dict:
    """Greedy peeling (Algorithm 3) on the GPU (lowd_greedy_peel): removal
    order, |E(S)| after each removal, S* and its density num/den."""
    torch = _torch()
    s = _dev(src, torch.int32, "src")
    d = _dev(dst, torch.int32, "dst")
    order = torch.empty(n, dtype=torch.int32, device=s.device)
    rem_m = torch.empty(n, dtype=torch.int64, device=s.device)
    in_set = torch.empty(n, dtype=torch.uint8, device=s.device)
    num, den = C.c_int64(0), C.c_int64(0)
    _check(lib().lowd_greedy_peel(n, s.numel(), _ptr(s), _ptr(d), _ptr(order), _ptr(rem_m),
                                  _ptr(in_set), C.byref(num), C.byref(den), _stream(stream)))
    return dict(order=order, rem_m=rem_m, in_set=in_set, num=int(num.value), den=int(den.value))


def densest_after_prune(n: int, src, dst, solver: str = "lowd", stream=None, **kw) -> dict:
    """Algorithm 2 with a plug-in DSPSolver: prune G, solve the pruned graph
    H with `solver` ("lowd" to a gap, or "greedy"), and map the set back to
    G's node ids.  Returns num/den (|E(S)|, |S|) and in_set over G."""
    torch = _torch()
    pr = prune(n, src, dst, stream)
    if pr["n_h"] == 0:
        raise LowdError(-2, "the pruned graph is empty")
    if solver == "lowd":
        r = solve(pr["n_h"], pr["src"].clone(), pr["dst"].clone(), None, stream=stream, **kw)
        sub = r["in_set"]
        out = dict(num=r["num"], den=r["den"], gap=r["gap"], sweeps=r["sweeps"])
    elif solver == "greedy":
        r = greedy_peel(pr["n_h"], pr["src"].clone(), pr["dst"].clone(), stream)
        sub = r["in_set"]
        out = dict(num=r["num"], den=r["den"])
    else:
        raise ValueError(solver)
    keep = pr["node_keep"].bool()
    in_set = torch.zeros(n, dtype=torch.uint8, device=keep.device)
    in_set[keep] = sub
    out.update(in_set=in_set, n_h=pr["n_h"], m_h=pr["m_h"], rounds=pr["rounds"])
    return out


class Solver:
    """LOWD on one graph: schedule, fractions and loads live on the GPU."""

    def __init__(self, n: int, src, dst, w=None, state: str = "f64", star_max: int = 16,
                 stream=None):
        torch = _torch()
        self.n = int(n)
        s = _dev(src, torch.int32, "src")
        d = _dev(dst, torch.int32, "dst")
        ww = _dev(w, torch.float32, "w", allow_none=True)
        self.m = s.numel()
        self.device = s.device
        self.weighted = ww is not None
        self.state = state
        h = C.c_void_p()
        _check(lib().lowd_init_loads(self.n, self.m, _ptr(s), _ptr(d), _ptr(ww), _STATES[state],
                                     star_max, C.byref(h), _stream(stream)))
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().lowd_solver_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def reset(self, stream=None):
        """Back to the equal-split initial state (schedule kept)."""
        _check(lib().lowd_reset_loads(self._h, _stream(stream)))

    def iterate(self, sweeps: int = 1, stream=None):
        _check(lib().lowd_iterate(self._h, int(sweeps), _stream(stream)))

    def check(self, stream=None, kept: bool = False):
        """(D, sum of loads, sum of squared loads).  kept: from the loads as
        the solver keeps them (FP32K: an estimate of D, no recomputation from
        the fractions); otherwise exact."""
        D, s, s2 = C.c_double(), C.c_double(), C.c_double()
        f = lib().lowd_check_kept if kept else lib().lowd_check
        _check(f(self._h, C.byref(D), C.byref(s), C.byref(s2), _stream(stream)))
        return D.value, s.value, s2.value

    def resync(self, stream=None):
        """F32K: restart the carried loads from the FP64 loads of the stored
        fractions (lowd_resync_loads); no-op for F64."""
        _check(lib().lowd_resync_loads(self._h, _stream(stream)))

    def extract(self, stream=None, kept: bool = False) -> dict:
        """The densest prefix of the descending-load order; kept as for
        check (the set's density is exact either way)."""
        torch = _torch()
        in_set = torch.empty(self.n, dtype=torch.uint8, device=self.device)
        nu, nw, den, D, gap = C.c_int64(), C.c_double(), C.c_int64(), C.c_double(), C.c_double()
        f = lib().lowd_extract_densest_kept if kept else lib().lowd_extract_densest
        _check(f(self._h, _ptr(in_set), C.byref(nu), C.byref(nw), C.byref(den), C.byref(D),
                 C.byref(gap), _stream(stream)))
        return dict(in_set=in_set, num=int(nu.value), num_w=float(nw.value), den=int(den.value),
                    D=float(D.value), gap=float(gap.value))

    def solve(self, tol: float = 1e-6, max_sweeps: int = 10000, check_every: int = 10,
              stream=None) -> dict:
        """lowd_solve from the current state: in_set (device), num (|E(S)|
        for unit weights), num_w, den, D, gap, sweeps and converged."""
        torch = _torch()
        in_set = torch.empty(self.n, dtype=torch.uint8, device=self.device)
        nu, nw, den, D, gap = C.c_int64(), C.c_double(), C.c_int64(), C.c_double(), C.c_double()
        sw = C.c_int32()
        st = _check(lib().lowd_solve(self._h, float(tol), int(max_sweeps), int(check_every),
                                     _ptr(in_set), C.byref(nu), C.byref(nw), C.byref(den),
                                     C.byref(D), C.byref(gap), C.byref(sw), _stream(stream)))
        return dict(in_set=in_set, num=int(nu.value), num_w=float(nw.value), den=int(den.value),
                    D=float(D.value), gap=float(gap.value), sweeps=int(sw.value),
                    converged=st == 0)

    def ldd(self, stream=None) -> dict:
        """The locally-dense decomposition read from the current loads:
        level per node (device int32), level ends k_end and f_end (numpy)."""
        torch = _torch()
        level = torch.empty(self.n, dtype=torch.int32, device=self.device)
        k_end = torch.empty(self.n, dtype=torch.int64, device=self.device)
        f_end = torch.empty(self.n, dtype=torch.float64, device=self.device)
        nl = C.c_int64()
        _check(lib().lowd_ldd_readout(self._h, _ptr(level), _ptr(k_end), _ptr(f_end),
                                      C.byref(nl), _stream(stream)))
        L = int(nl.value)
        return dict(level=level, k_end=k_end[:L].cpu().numpy(), f_end=f_end[:L].cpu().numpy())

    def trace(self, sweeps: int, every: int = 1, stream=None) -> np.ndarray:
        """Continues `sweeps` sweeps, recording (sweeps, D, rho, sum_sq, gap)
        before the first and every `every` sweeps (lowd_convergence_trace)."""
        rows = (sweeps + every - 1) // every + 1
        out = np.zeros((rows, 5), dtype=np.float64)
        pts = C.c_int64()
        _check(lib().lowd_convergence_trace(self._h, sweeps, every,
                                            out.ctypes.data_as(C.c_void_p), C.byref(pts),
                                            _stream(stream)))
        return out[:pts.value]

    def read_state(self, stream=None):
        torch = _torch()
        x = torch.empty(max(self.m, 1), dtype=torch.float64, device=self.device)
        L = torch.empty(self.n, dtype=torch.float64, device=self.device)
        _check(lib().lowd_read_state(self._h, _ptr(x), _ptr(L), _stream(stream)))
        return x[:self.m], L

    def schedule(self):
        phase = np.zeros(max(self.m, 1), dtype=np.int32)
        center = np.zeros(max(self.m, 1), dtype=np.int32)
        P = C.c_int32()
        _check(lib().lowd_schedule_export(self._h, phase.ctypes.data_as(C.c_void_p),
                                          center.ctypes.data_as(C.c_void_p), C.byref(P)))
        return phase[:self.m], center[:self.m], int(P.value)

    def info(self) -> dict:
        a = np.zeros(12, dtype=np.int64)
        _check(lib().lowd_solver_info(self._h, a.ctypes.data_as(C.c_void_p)))
        keys = ["n", "m", "phases", "grid_phases", "mid_phases", "lds_phases", "lds_nodes",
                "lds_edges", "mid_edges", "state", "node_layout", "pulled_phases"]
        return {k: int(v) for k, v in zip(keys, a)}


LOWD_NOT_CONVERGED = 1


def solve(n: int, src, dst, w=None, state: str = "f64", star_max: int = 16, tol: float = 1e-6,
          check_every: int = 10, max_sweeps: int = 10000, stream=None) -> dict:
    """A new solver for the graph, then lowd_solve: sweeps until the density
    gap (D - rho) / rho is at most `tol` (Section III-B's bounds) or
    max_sweeps.  Returns the dict of Solver.solve plus the solver itself."""
    sv = Solver(n, src, dst, w, state, star_max, stream)
    ex = sv.solve(tol, max_sweeps, check_every, stream)
    ex["solver"] = sv
    return ex


def batch_solve(graphs, tol: float = 1e-6, state: str = "f64", star_max: int = 16,
                max_sweeps: int = 20000, check_every: int = 10, stream=None) -> dict:
    """Many unweighted graphs (each with .n, .src, .dst in local ids), each
    solved to a certified gap `tol` (lowd_batch_solve).  Returns per-graph
    num/den/D/sweeps (numpy), the concatenated in_set (device tensor), node
    and edge offsets, and whether every graph converged."""
    torch = _torch()
    G = len(graphs)
    node_ptr, edge_ptr, src, dst = _batch_arrays(graphs)
    N = int(node_ptr[-1])
    in_set = torch.empty(max(N, 1), dtype=torch.uint8, device=src.device)
    num = torch.empty(G, dtype=torch.int64, device=src.device)
    den = torch.empty(G, dtype=torch.int64, device=src.device)
    D = torch.empty(G, dtype=torch.float64, device=src.device)
    used = torch.empty(G, dtype=torch.int32, device=src.device)
    at = torch.empty(G, dtype=torch.int32, device=src.device)
    st = _check(lib().lowd_batch_solve(G, node_ptr.ctypes.data_as(C.c_void_p),
                                       edge_ptr.ctypes.data_as(C.c_void_p), _ptr(src), _ptr(dst),
                                       _STATES[state], star_max, float(tol), int(max_sweeps),
                                       int(check_every), _ptr(in_set), _ptr(num), _ptr(den),
                                       _ptr(D), _ptr(used), _ptr(at), _stream(stream)))
    return dict(num=num.cpu().numpy(), den=den.cpu().numpy(), D=D.cpu().numpy(),
                sweeps=used.cpu().numpy(), set_sweeps=at.cpu().numpy(), in_set=in_set[:N],
                node_ptr=node_ptr, edge_ptr=edge_ptr, converged=st == 0)


def batch_run(graphs, sweeps: int, state: str = "f64", star_max: int = 16, stream=None) -> dict:
    """A fixed number of sweeps on every graph of a batch (lowd_batch_prepare,
    lowd_batch_iterate, lowd_batch_extract): per-graph num/den (numpy), the
    concatenated in_set and FP64 loads (device), node and edge offsets."""
    b = Batch(graphs, state, star_max, stream=stream)
    b.iterate(sweeps, stream)
    b.extract(stream, loads=True)
    out = dict(num=b.num.cpu().numpy(), den=b.den.cpu().numpy(), in_set=b.in_set.clone(),
               load=b.load.clone(), D=b.D.cpu().numpy(), node_ptr=b.node_ptr,
               edge_ptr=b.edge_ptr)
    b.close()
    return out


def dks_bound(k_end: np.ndarray, f_end: np.ndarray, k: int) -> float:
    """Corollary 1 (lowd_dks_bound): upper bound on the density of any
    k-node subgraph from a decomposition read-out (Solver.ldd())."""
    ke = np.ascontiguousarray(k_end, dtype=np.int64)
    fe = np.ascontiguousarray(f_end, dtype=np.float64)
    b = C.c_double()
    _check(lib().lowd_dks_bound(ke.ctypes.data_as(C.c_void_p), fe.ctypes.data_as(C.c_void_p),
                                ke.size, int(k), C.byref(b)))
    return b.value


def _batch_arrays(graphs):
    torch = _torch()
    G = len(graphs)
    node_ptr = np.zeros(G + 1, dtype=np.int64)
    edge_ptr = np.zeros(G + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        node_ptr[i + 1] = node_ptr[i] + g.n
        edge_ptr[i + 1] = edge_ptr[i] + g.src.size
    src = torch.from_numpy(np.concatenate([g.src for g in graphs]).astype(np.int32)).cuda()
    dst = torch.from_numpy(np.concatenate([g.dst for g in graphs]).astype(np.int32)).cuda()
    return node_ptr, edge_ptr, src, dst


class Batch:
    """A prepared batch of unweighted graphs (lowd_batch_prepare): iterate in
    steps and extract every graph's densest set and dual bound D_g."""

    def __init__(self, graphs, state: str = "f64", star_max: int = 16, tune: bool = False,
                 stream=None):
        torch = _torch()
        self.G = len(graphs)
        self.node_ptr, self.edge_ptr, src, dst = _batch_arrays(graphs)
        self.N = int(self.node_ptr[-1])
        self.device = src.device
        h = C.c_void_p()
        _check(lib().lowd_batch_prepare(self.G, self.node_ptr.ctypes.data_as(C.c_void_p),
                                        self.edge_ptr.ctypes.data_as(C.c_void_p), _ptr(src),
                                        _ptr(dst), _STATES[state], star_max, 1 if tune else 0,
                                        C.byref(h), _stream(stream)))
        self._h = h
        self.in_set = torch.empty(self.N, dtype=torch.uint8, device=self.device)
        self.num = torch.empty(self.G, dtype=torch.int64, device=self.device)
        self.den = torch.empty(self.G, dtype=torch.int64, device=self.device)
        self.D = torch.empty(self.G, dtype=torch.float64, device=self.device)
        self.load = torch.empty(self.N, dtype=torch.float64, device=self.device)

    def reset(self, stream=None):
        _check(lib().lowd_batch_reset(self._h, _stream(stream)))

    def iterate(self, sweeps: int, stream=None):
        _check(lib().lowd_batch_iterate(self._h, sweeps, _stream(stream)))

    def extract(self, stream=None, loads: bool = False):
        """Enqueues the extraction into self.in_set/num/den/D (and self.load)."""
        _check(lib().lowd_batch_extract(self._h, _ptr(self.in_set), _ptr(self.num),
                                        _ptr(self.den), _ptr(self.D),
                                        _ptr(self.load) if loads else None, _stream(stream)))

    def retire(self, tol: float, stream=None):
        """Stops iterating the graphs whose gap after the last extract() is at
        most tol; returns (graphs still iterating, their edges)."""
        a = C.c_int32()
        ae = C.c_int64()
        _check(lib().lowd_batch_retire(self._h, _ptr(self.num), _ptr(self.den), _ptr(self.D),
                                       float(tol), C.byref(a), C.byref(ae), _stream(stream)))
        return a.value, ae.value

    def solve(self, tol: float = 1e-6, max_sweeps: int = 20000, check_every: int = 10,
              stream=None) -> dict:
        """lowd_batch_solve_prepared from the current state into self.in_set,
        num, den, D; returns per-graph sweeps, the sweep count of each set's
        extraction (numpy) and whether every graph converged."""
        torch = _torch()
        used = torch.empty(self.G, dtype=torch.int32, device=self.device)
        at = torch.empty(self.G, dtype=torch.int32, device=self.device)
        st = _check(lib().lowd_batch_solve_prepared(self._h, float(tol), int(max_sweeps),
                                                    int(check_every), _ptr(self.in_set),
                                                    _ptr(self.num), _ptr(self.den), _ptr(self.D),
                                                    _ptr(used), _ptr(at), _stream(stream)))
        return dict(sweeps=used.cpu().numpy(), set_sweeps=at.cpu().numpy(), converged=st == 0)

    def gaps(self):
        """Per-graph relative gap (D_g - rho_g) / rho_g after extract()."""
        num = self.num.cpu().numpy().astype(np.float64)
        den = self.den.cpu().numpy().astype(np.float64)
        D = self.D.cpu().numpy()
        rho = num / den
        with np.errstate(divide="ignore", invalid="ignore"):
            gap = np.where(rho > 0, (D - rho) / rho, np.where(D > 0, np.inf, 0.0))
        return gap

    def info(self) -> dict:
        a = np.zeros(9, dtype=np.int64)
        _check(lib().lowd_batch_info(self._h, a.ctypes.data_as(C.c_void_p)))
        keys = ["G", "N", "M", "phases", "max_phases", "waves", "prefetch", "blocks", "lds"]
        return {k: int(v) for k, v in zip(keys, a)}

    def close(self):
        if getattr(self, "_h", None):
            lib().lowd_batch_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def schedule_build(n: int, src: np.ndarray, dst: np.ndarray, star_max: int = 16):
    """The phase schedule computed on the host (no GPU needed):
    (phase int32[m], center int32[m], nphases)."""
    src = np.ascontiguousarray(src, dtype=np.int32)
    dst = np.ascontiguousarray(dst, dtype=np.int32)
    m = src.size
    phase = np.zeros(max(m, 1), dtype=np.int32)
    center = np.zeros(max(m, 1), dtype=np.int32)
    P = C.c_int32()
    _check(lib().lowd_schedule_build(n, m, src.ctypes.data_as(C.c_void_p),
                                     dst.ctypes.data_as(C.c_void_p), star_max,
                                     phase.ctypes.data_as(C.c_void_p),
                                     center.ctypes.data_as(C.c_void_p), C.byref(P)))
    return phase[:m], center[:m], int(P.value)


def version() -> str:
    return lib().lowd_version().decode()
