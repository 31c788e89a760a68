// api.hip -- the C interface (include/lowd.h): argument checks, the solver
// object, device memory, the HIP graph of one sweep, and error reporting.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <exception>
#include <thread>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "extract.h"
#include "lowd_internal.h"
#include "prune.h"
#include "sweep_state.h"
#include "wg_check.h"

namespace lowd {

static thread_local std::string g_last_error;

void fail(int32_t status, const std::string &msg) { throw Error{status, msg}; }

void hip_check(hipError_t e, const char *what) {
    if (e == hipSuccess) return;
    int32_t st = (e == hipErrorOutOfMemory) ? LOWD_E_NOMEM : LOWD_E_HIP;
    fail(st, std::string(what) + ": " + hipGetErrorString(e));
}

template <class F>
static lowd_status guarded(F &&f) {
    g_last_error.clear();
    try {
        f();
        return LOWD_OK;
    } catch (const Error &e) {
        g_last_error = e.msg;
        return e.status;
    } catch (const std::bad_alloc &) {
        g_last_error = "host allocation failed";
        return LOWD_E_NOMEM;
    } catch (const std::exception &e) {
        g_last_error = e.what();
        return LOWD_E_ARG;
    } catch (...) {
        g_last_error = "unknown error";
        return LOWD_E_ARG;
    }
}

template <class T>
static void upload(DBuf<T> &d, const std::vector<T> &h, hipStream_t s) {
    d.alloc(h.size());
    if (!h.empty())
        LOWD_HIP(hipMemcpyAsync(d.p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, s));
}

static size_t lds_capacity_bytes() {
    int dev = 0, v = 0;
    LOWD_HIP(hipGetDevice(&dev));
    LOWD_HIP(hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    size_t cap = (size_t)v;
    if (cap > 160 * 1024) cap = 160 * 1024;
    return cap;
}

// Checks the edge list on the device (ids in range, no self-loop, weights
// positive and finite, no repeated pair) and fails with the first bad edge.
// Its device buffers come from `ws` and are released on return; a region
// without a base only measures them.
static void validate_graph_ws(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                              const float *w, Arena &ws, hipStream_t s) {
    int64_t invalid = -1;
    const int64_t b = find_duplicate_pair_ws(n, m, src, dst, ws, s, w, &invalid);
    const bool repeated = invalid < 0;
    const int64_t at = repeated ? b : invalid;
    if (at >= 0) {
        int32_t a = 0, c = 0;
        float x = 1.0f;
        LOWD_HIP(hipMemcpyAsync(&a, src + at, 4, hipMemcpyDeviceToHost, s));
        LOWD_HIP(hipMemcpyAsync(&c, dst + at, 4, hipMemcpyDeviceToHost, s));
        if (w) LOWD_HIP(hipMemcpyAsync(&x, w + at, 4, hipMemcpyDeviceToHost, s));
        LOWD_HIP(hipStreamSynchronize(s));
        fail(LOWD_E_GRAPH, std::string(repeated ? "repeated pair" : "invalid edge") +
                               " at index " + std::to_string(at) + ": (" + std::to_string(a) +
                               ", " + std::to_string(c) + ") weight " + std::to_string(x) +
                               " (n = " + std::to_string(n) + ")");
    }
}

static size_t validate_ws_bytes(int32_t n, int64_t m, const float *w) {
    Arena measure;
    validate_graph_ws(n, m, nullptr, nullptr, w, measure, nullptr);
    return measure.peak;
}

static void validate_graph(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                           const float *w, hipStream_t s) {
    DBuf<char> buf(validate_ws_bytes(n, m, w));
    Arena ws(buf.p, buf.bytes());
    validate_graph_ws(n, m, src, dst, w, ws, s);
}

// Where a node's load waits between phases: at its next station (the
// default), or in one node-indexed array (LOWD_LAYOUT=node).  The array is
// small enough for the on-die caches, but a tile then reads its leaf ids
// before it can gather their loads (two dependent round trips instead of
// one), and the gathers are random: on uniform random graphs with wide
// phases (2^22 nodes and 2^28 edges; 2^19 and 2^27, whose array fits each
// L2) a sweep took 1.5 times as long as with stations, so stations are the
// default everywhere.
static bool choose_node_layout() {
    if (const char *e = getenv("LOWD_LAYOUT")) {
        if (!strcmp(e, "node")) return true;
        if (!strcmp(e, "station")) return false;
        fail(LOWD_E_ARG, "LOWD_LAYOUT must be node or station");
    }
    return false;
}

}  // namespace lowd

using namespace lowd;

struct lowd_solver {
    int32_t n = 0;
    int64_t m = 0;
    int32_t state = 0;
    bool weighted = false;
    Schedule sch;
    SweepLaunch fn{};
    // device copies of the graph (for extraction and read-out)
    DBuf<int32_t> e_src, e_dst;
    DBuf<float> e_w;
    // weighted: each weight over 2^wq as an exact integer (the extraction's
    // densities are decided exactly)
    DBuf<uint64_t> e_wi;
    DBuf<uint64_t> e_wi_inc;   // [2m] weighted: e_wi of each incidence entry's edge
    int32_t wq = 0;
    Csr csr;
    // schedule layout
    DBuf<int32_t> tile_center;
    DBuf<PhaseDesc> tail_desc, mid_desc;
    DBuf<int64_t> slot_edge, edge_slot;
    DBuf<uint32_t> slot_leaf, slot_next, center_next, tail_next, home;
    DBuf<uint32_t> slot_src, center_src;   // pulled phases' sources (empty: none)
    // state: fractions per slot, loads at their stations
    DBuf<char> slot_x, E;
    DBuf<float> slot_w;
    DBuf<double> L64, stats_partial, stats_out;
    ExtractScratch ex;
    LddScratch ldd;
    DBuf<uint8_t> ldd_in_set;
    DBuf<uint8_t> solve_in_set;   // lowd_solve: each check's extraction
    // the other end of each incidence entry, and the nodes of degree >=
    // kBigRow, for the per-node kernels (initial loads, recompute, extraction)
    DBuf<int32_t> adj, big;
    int32_t nbig = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t ntail = 0;
    int64_t nslots = 0;
    // loads in a node-indexed array (wide phases) instead of at stations
    bool node_layout = false;
    ~lowd_solver() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

static void reset_state(lowd_solver *sv, hipStream_t s) {
    const int64_t nslots = sv->nslots;
    if (nslots > 0)
        sv->fn.init_slots(nslots, sv->slot_edge.p, sv->weighted ? sv->e_w.p : nullptr,
                          sv->slot_x.p, sv->weighted ? sv->slot_w.p : nullptr, s);
    if (sv->node_layout) sv->fn.fill_nodes(sv->n, sv->E.p, s);
    sv->fn.init_loads(sv->n, sv->csr.row_ptr.p, sv->csr.inc.p, sv->weighted ? sv->e_w.p : nullptr,
                      sv->home.p, sv->big.p, sv->nbig, sv->node_layout ? 0 : sv->sch.entries,
                      sv->sch.center_base, sv->E.p, s);
    LOWD_HIP(hipGetLastError());
}

extern "C" {

const char *lowd_version(void) { return "lowd-gfx950 0.1"; }

const char *lowd_last_error(void) { return g_last_error.c_str(); }

lowd_status lowd_init_loads(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                            const float *w, int32_t state, int32_t star_max, lowd_solver **out,
                            void *stream) {
    return guarded([&] {
        if (!out) fail(LOWD_E_ARG, "out is NULL");
        *out = nullptr;
        if (n < 1 || n > 0x7FFFFFFD) fail(LOWD_E_ARG, "n must be in [1, 2^31 - 3]");
        if (m < 0 || m >= ((int64_t)1 << 31)) fail(LOWD_E_ARG, "m must be in [0, 2^31)");
        if (m > 0 && (!src || !dst)) fail(LOWD_E_ARG, "src/dst is NULL");
        if (state != LOWD_STATE_F64 && state != LOWD_STATE_F32K) fail(LOWD_E_ARG, "bad state");
        if (star_max < 1 || star_max > kMaxStar) fail(LOWD_E_ARG, "star_max must be in [1, 32]");
        hipStream_t s = (hipStream_t)stream;
        validate_graph(n, m, src, dst, w, s);

        auto sv = new lowd_solver();
        std::unique_ptr<lowd_solver> guard(sv);
        sv->n = n;
        sv->m = m;
        sv->state = state;
        sv->weighted = w != nullptr;
        get_sweep_launchers(state, sv->weighted, sv->fn);

        // host copy of the edge list for the schedule
        std::vector<int32_t> hs((size_t)m), hd((size_t)m);
        if (m > 0) {
            LOWD_HIP(hipMemcpyAsync(hs.data(), src, (size_t)m * 4, hipMemcpyDeviceToHost, s));
            LOWD_HIP(hipMemcpyAsync(hd.data(), dst, (size_t)m * 4, hipMemcpyDeviceToHost, s));
            LOWD_HIP(hipStreamSynchronize(s));
        }
        sv->node_layout = choose_node_layout();
        const int64_t lds = sv->node_layout ? 0 : (int64_t)lds_capacity_bytes();
        int64_t force0 = -1, force1 = -1, pull_edges = -1;
        if (!sv->node_layout) {
            if (const char *e = getenv("LOWD_TAIL_SPLIT")) force0 = atoll(e);
            if (const char *e = getenv("LOWD_MID_SPLIT")) force1 = atoll(e);
            // whole-GPU phases this wide gather their loads (random reads)
            // instead of scattering them (random writes, half the rate)
            pull_edges = kPullMinEdges;
            if (const char *e = getenv("LOWD_PULL_EDGES")) pull_edges = atoll(e);
        }
        build_schedule(n, m, hs.data(), hd.data(), star_max, lds, (int64_t)sv->fn.l_bytes, force0,
                       force1, sv->sch, false, pull_edges);
        const Schedule &sc = sv->sch;

        // device copies of the graph, incidence rows
        sv->e_src.alloc((size_t)m);
        sv->e_dst.alloc((size_t)m);
        if (m > 0) {
            LOWD_HIP(hipMemcpyAsync(sv->e_src.p, src, (size_t)m * 4, hipMemcpyDeviceToDevice, s));
            LOWD_HIP(hipMemcpyAsync(sv->e_dst.p, dst, (size_t)m * 4, hipMemcpyDeviceToDevice, s));
        }
        if (sv->weighted) {
            sv->e_w.alloc((size_t)m);
            if (m > 0)
                LOWD_HIP(
                    hipMemcpyAsync(sv->e_w.p, w, (size_t)m * 4, hipMemcpyDeviceToDevice, s));
            sv->e_wi.alloc((size_t)m);
            DBuf<int32_t> range(2);
            fixed_point_weights(m, sv->e_w.p, sv->e_wi.p, &sv->wq, range.p, s);
        }
        build_incidence(n, m, sv->e_src.p, sv->e_dst.p, sv->csr, s);
        if (sv->weighted) {
            sv->e_wi_inc.alloc((size_t)(2 * m));
            build_entry_weights(m, sv->csr.inc.p, sv->e_wi.p, sv->e_wi_inc.p, s);
        }
        {
            sv->adj.alloc((size_t)(2 * m));
            build_adjacency(m, sv->csr, sv->e_src.p, sv->e_dst.p, sv->adj.p, s);
            // the nodes of degree >= kBigRow, from the incidence rows' offsets
            std::vector<int64_t> rp((size_t)n + 1);
            LOWD_HIP(hipMemcpyAsync(rp.data(), sv->csr.row_ptr.p, rp.size() * sizeof(int64_t),
                                    hipMemcpyDeviceToHost, s));
            LOWD_HIP(hipStreamSynchronize(s));
            std::vector<int32_t> big;
            for (int32_t u = 0; u < n; ++u)
                if (rp[(size_t)u + 1] - rp[(size_t)u] >= kBigRow) big.push_back(u);
            upload(sv->big, big, s);
            sv->nbig = (int32_t)big.size();
        }

        // schedule layout
        upload(sv->tile_center, sc.tile_center, s);
        upload(sv->slot_leaf, sc.slot_leaf, s);
        upload(sv->slot_edge, sc.slot_edge, s);
        upload(sv->edge_slot, sc.edge_slot, s);
        // the single-workgroup tiers stage their descriptors in LDS in the
        // narrow form (their phases are at most kTierStar deep)
        std::vector<PhaseDesc> tdesc, mdesc;
        for (int32_t p = sc.P0; p < sc.P; ++p) tdesc.push_back(narrow_desc<kTierStar>(sc.desc[(size_t)p]));
        for (int32_t p = sc.P1; p < sc.P0; ++p) mdesc.push_back(narrow_desc<kTierStar>(sc.desc[(size_t)p]));
        upload(sv->tail_desc, tdesc, s);
        upload(sv->mid_desc, mdesc, s);
        if (sv->node_layout) {
            // a node's load lives at its own index
            std::vector<uint32_t> home((size_t)n);
            for (int32_t u = 0; u < n; ++u) home[(size_t)u] = (uint32_t)u;
            upload(sv->home, home, s);
        } else {
            upload(sv->slot_next, sc.slot_next, s);
            upload(sv->center_next, sc.center_next, s);
            upload(sv->tail_next, sc.tail_next, s);
            upload(sv->home, sc.home, s);
            if (!sc.pull.empty()) {
                upload(sv->slot_src, sc.slot_src, s);
                upload(sv->center_src, sc.center_src, s);
            }
        }
        sv->ntail = (int32_t)sc.tail_nodes.size();

        // state
        const int64_t nslots = (int64_t)sc.slot_leaf.size();
        sv->nslots = nslots;
        sv->slot_x.alloc((size_t)nslots * sv->fn.x_bytes);
        if (sv->weighted) sv->slot_w.alloc((size_t)nslots);
        sv->E.alloc((size_t)(sv->node_layout ? (int64_t)n + 2 : sc.entries) * sv->fn.l_bytes);
        sv->L64.alloc((size_t)n);
        sv->stats_partial.alloc(3 * 1024);
        sv->stats_out.alloc(3);
        reset_state(sv, s);

        // one sweep as a HIP graph: a kernel per whole-GPU phase, then the
        // LDS-resident workgroup for the last phases
        if (sc.P > 0) {
            size_t tail_lds =
                tail_desc_bytes(sc.P - sc.P0) + ((size_t)sv->ntail + 2) * sv->fn.l_bytes;
            if (sc.P0 < sc.P) sv->fn.set_tail_lds(tail_lds);
            if (sc.P1 < sc.P0) sv->fn.set_mid_lds(tail_desc_bytes(sc.P0 - sc.P1));
            hipStream_t cs;
            LOWD_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            hipError_t err = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (err == hipSuccess) {
                const float *sw = sv->weighted ? sv->slot_w.p : nullptr;
                for (int32_t p = 0; p < sc.P1; ++p) {
                    if (sv->node_layout)
                        sv->fn.phase_node(sc.desc[(size_t)p], sv->tile_center.p, sv->slot_leaf.p,
                                          sv->slot_x.p, sw, sv->E.p, cs);
                    else {
                        const bool pull = !sc.pull.empty() && sc.pull[(size_t)p];
                        sv->fn.phase(sc.desc[(size_t)p], sc.center_base, sv->center_next.p,
                                     sv->slot_next.p, sv->slot_x.p, sw, sv->E.p,
                                     pull ? sv->slot_src.p : nullptr,
                                     pull ? sv->center_src.p : nullptr, cs);
                    }
                }
                if (sc.P1 < sc.P0)
                    sv->fn.mid(sc.P0 - sc.P1, sv->mid_desc.p, sc.center_base, sv->center_next.p,
                               sv->slot_next.p, sv->slot_x.p, sw, sv->E.p, cs);
                if (sc.P0 < sc.P)
                    sv->fn.tail(sc.P - sc.P0, sv->tail_desc.p, sv->tile_center.p,
                                sv->slot_leaf.p, sv->slot_x.p, sw, sc.tail_base,
                                sv->tail_next.p, sv->ntail, sv->E.p, cs);
                err = hipStreamEndCapture(cs, &sv->graph);
            }
            (void)hipStreamDestroy(cs);
            LOWD_HIP(err);
            LOWD_HIP(hipGraphInstantiate(&sv->exec, sv->graph, nullptr, nullptr, 0));
        }
        LOWD_HIP(hipStreamSynchronize(s));
        // the layout lives on the device now; keep only what later calls read
        // (phases and centers for lowd_schedule_export, counts for info)
        {
            Schedule &k = sv->sch;
            std::vector<int32_t>().swap(k.tile_center);
            std::vector<uint32_t>().swap(k.slot_leaf);
            std::vector<int64_t>().swap(k.slot_edge);
            std::vector<int64_t>().swap(k.edge_slot);
            std::vector<int32_t>().swap(k.tail_nodes);
            std::vector<uint32_t>().swap(k.slot_next);
            std::vector<uint32_t>().swap(k.center_next);
            std::vector<uint32_t>().swap(k.tail_next);
            std::vector<uint32_t>().swap(k.home);
        }
        *out = guard.release();
    });
}

lowd_status lowd_reset_loads(lowd_solver *sv, void *stream) {
    return guarded([&] {
        if (!sv) fail(LOWD_E_ARG, "solver is NULL");
        reset_state(sv, (hipStream_t)stream);
    });
}

lowd_status lowd_iterate(lowd_solver *sv, int32_t sweeps, void *stream) {
    return guarded([&] {
        if (!sv) fail(LOWD_E_ARG, "solver is NULL");
        if (sweeps < 0) fail(LOWD_E_ARG, "sweeps must be >= 0");
        if (!sv->exec) return;
        for (int32_t t = 0; t < sweeps; ++t) LOWD_HIP(hipGraphLaunch(sv->exec, (hipStream_t)stream));
    });
}

// FP64 loads into L64: for LOWD_STATE_F32K recomputed from the fractions
// (exact), or the kept compensated pairs rounded to FP64 (kept)
static void loads_f64(lowd_solver *sv, hipStream_t s, bool kept = false) {
    if (kept) {
        sv->fn.read_loads(sv->n, sv->home.p, sv->E.p, sv->L64.p, s);
        return;
    }
    sv->fn.loads_f64(sv->n, sv->csr.row_ptr.p, sv->csr.inc.p, sv->edge_slot.p, sv->slot_x.p,
                     sv->weighted ? sv->e_w.p : nullptr, sv->home.p, sv->big.p, sv->nbig, sv->E.p,
                     sv->L64.p, s);
}

static void stats(lowd_solver *sv, double out[3], hipStream_t s) {
    int32_t nb = (int32_t)grid_for(sv->n, 256, 1024);
    launch_stats(sv->n, sv->L64.p, sv->stats_partial.p, nb, sv->stats_out.p, s);
    LOWD_HIP(hipGetLastError());
    LOWD_HIP(hipMemcpyAsync(out, sv->stats_out.p, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    LOWD_HIP(hipStreamSynchronize(s));
}

static void check_impl(lowd_solver *sv, bool kept, double *D, double *sum_loads,
                       double *sum_sq_loads, hipStream_t s) {
    if (!sv) fail(LOWD_E_ARG, "solver is NULL");
    loads_f64(sv, s, kept);
    double o[3];
    stats(sv, o, s);
    if (D) *D = o[0];
    if (sum_loads) *sum_loads = o[1];
    if (sum_sq_loads) *sum_sq_loads = o[2];
}

static void extract_api(lowd_solver *sv, bool kept, uint8_t *in_set, int64_t *num_unit,
                        double *num_w, int64_t *den, double *D, double *gap, hipStream_t s,
                        u128 *w_exact = nullptr) {
    if (!sv) fail(LOWD_E_ARG, "solver is NULL");
    if (!in_set) fail(LOWD_E_ARG, "in_set is NULL");
    loads_f64(sv, s, kept);
    ExtractArgs a;
    a.n = sv->n;
    a.m = sv->m;
    a.weighted = sv->weighted;
    a.L64 = sv->L64.p;
    a.row_ptr = sv->csr.row_ptr.p;
    a.inc = sv->csr.inc.p;
    a.src = sv->e_src.p;
    a.dst = sv->e_dst.p;
    a.w = sv->weighted ? sv->e_w.p : nullptr;
    a.wi = sv->weighted ? sv->e_wi.p : nullptr;
    a.wi_inc = sv->weighted ? sv->e_wi_inc.p : nullptr;
    a.wq = sv->wq;
    if (sv->m > 0) {
        a.adj = sv->adj.p;
        a.big = sv->big.p;
        a.nbig = sv->nbig;
    }
    a.in_set = in_set;
    launch_extract(a, sv->ex, s);
    int64_t best[3];
    LOWD_HIP(hipMemcpyAsync(best, sv->ex.best.p, sizeof(best), hipMemcpyDeviceToHost, s));
    double o[3];
    stats(sv, o, s);   // synchronises
    int64_t dn = (int64_t)sv->n - best[0];
    double wnum;
    if (sv->weighted) {
        u128 wi;
        memcpy(&wi, &best[1], sizeof(wi));
        if (w_exact) *w_exact = wi;
        wnum = std::ldexp(u128_to_double(wi), sv->wq);   // rounded once
    } else {
        wnum = (double)best[1];
        if (w_exact) *w_exact = (u128)best[1];
    }
    if (num_unit) *num_unit = sv->weighted ? 0 : best[1];
    if (num_w) *num_w = wnum;
    if (den) *den = dn;
    if (D) *D = o[0];
    double rho = wnum / (double)dn;
    if (gap) *gap = rho > 0.0 ? (o[0] - rho) / rho : (o[0] > 0.0 ? 1.0e300 : 0.0);
}

lowd_status lowd_check(lowd_solver *sv, double *D, double *sum_loads, double *sum_sq_loads,
                       void *stream) {
    return guarded([&] { check_impl(sv, false, D, sum_loads, sum_sq_loads, (hipStream_t)stream); });
}

lowd_status lowd_resync_loads(lowd_solver *sv, void *stream) {
    return guarded([&] {
        if (!sv) fail(LOWD_E_ARG, "solver is NULL");
        if (sv->state != LOWD_STATE_F32K || sv->m == 0) return;
        hipStream_t s = (hipStream_t)stream;
        loads_f64(sv, s, false);
        sv->fn.write_loads(sv->n, sv->home.p, sv->L64.p, sv->E.p, s);
        LOWD_HIP(hipGetLastError());
    });
}

lowd_status lowd_check_kept(lowd_solver *sv, double *D, double *sum_loads, double *sum_sq_loads,
                            void *stream) {
    return guarded([&] { check_impl(sv, true, D, sum_loads, sum_sq_loads, (hipStream_t)stream); });
}

lowd_status lowd_extract_densest(lowd_solver *sv, uint8_t *in_set, int64_t *num_unit,
                                 double *num_w, int64_t *den, double *D, double *gap,
                                 void *stream) {
    return guarded([&] {
        extract_api(sv, false, in_set, num_unit, num_w, den, D, gap, (hipStream_t)stream);
    });
}

lowd_status lowd_extract_densest_kept(lowd_solver *sv, uint8_t *in_set, int64_t *num_unit,
                                      double *num_w, int64_t *den, double *D, double *gap,
                                      void *stream) {
    return guarded([&] {
        extract_api(sv, true, in_set, num_unit, num_w, den, D, gap, (hipStream_t)stream);
    });
}

// ------------------------------------------------------------ solve ------
// The stopping rule of Section III-B.  The largest load D bounds the maximum
// density from above at every sweep (weak duality), and the density of any
// extracted set bounds it from below, so the densest set extracted so far is
// certified once (D - rho_best) / rho_best <= tol.
}  // extern "C"

namespace {

struct Extracted {
    bool have = false;
    int64_t num_unit = 0;   // |E(S)| (unit weights)
    double num_w = 0.0;     // W(S) in FP64
    u128 w_exact = 0;       // W(S) exactly (weighted: in units of 2^wq)
    int64_t den = 0;        // |S|
};

double relative_gap(double D, double rho) {
    return rho > 0.0 ? (D - rho) / rho : (D > 0.0 ? 1.0e300 : 0.0);
}

double density_of(const Extracted &x) {
    return x.den > 0 ? x.num_w / (double)x.den : 0.0;
}

// a at least as dense as b, exactly by cross-multiplication (W < 2^95 in
// units of 2^wq, |S| < 2^31: the products stay below 2^126)
bool at_least_as_dense(const Extracted &a, const Extracted &b) {
    return a.w_exact * (u128)b.den >= b.w_exact * (u128)a.den;
}

// Sweeps before the next check.  From the last two (sweeps, gap) records:
// the gap decays about geometrically, so they predict when it reaches tol
// (at least 1, at most check_every).  Without such a prediction (the first
// checks, or a gap that did not fall): the sweeps done so far, so that check
// points double, but at least k_min and at most check_every; the first check
// comes after one sweep.
int32_t next_check(const std::vector<std::pair<int64_t, double>> &hist, double tol,
                   int32_t check_every, int32_t k_min) {
    if (hist.size() >= 2) {
        const auto &a = hist[hist.size() - 2];
        const auto &b = hist[hist.size() - 1];
        const double g0 = a.second, g1 = b.second;
        if (g1 > 0.0 && g1 < g0 && b.first > a.first && g1 > tol) {
            const double rate = std::pow(g1 / g0, 1.0 / (double)(b.first - a.first));
            if (rate < 1.0) {
                const double k = std::ceil(std::log(tol / g1) / std::log(rate));
                return (int32_t)std::max(1.0, std::min(k, (double)check_every));
            }
        }
    }
    if (hist.empty()) return 1;
    const int64_t done = hist.back().first;
    return (int32_t)std::max<int64_t>(1, std::min<int64_t>(std::max<int64_t>(k_min, done),
                                                           check_every));
}

}  // namespace

// One convergence check.  D alone is cheap; the extraction (a sort of every
// node) runs only when D does not already certify the best set.  Both read
// the loads as kept; for LOWD_STATE_F32K those only follow the loads of the
// stored fractions, so a gap within tol is confirmed with the exact D
// (recomputed from the fractions) before it counts, and when the exact D
// fails where the kept one passed, the carried loads restart from the
// fractions' loads.  Returns the gap of the best set; *D_out is the D it
// was taken with.
static double certify(lowd_solver *sv, Extracted &best, uint8_t *best_in_set, double tol,
                      double *D_out, hipStream_t s) {
    const bool exact = sv->state == LOWD_STATE_F64;
    auto confirm = [&](double D, double gap) {
        if (gap <= tol && !exact) {
            check_impl(sv, false, &D, nullptr, nullptr, s);
            gap = relative_gap(D, density_of(best));
            if (gap > tol) {
                loads_f64(sv, s, false);
                sv->fn.write_loads(sv->n, sv->home.p, sv->L64.p, sv->E.p, s);
                LOWD_HIP(hipGetLastError());
            }
        }
        *D_out = D;
        return gap;
    };
    if (best.have) {
        double D = 0.0;
        check_impl(sv, true, &D, nullptr, nullptr, s);
        const double gap = relative_gap(D, density_of(best));
        if (gap <= tol) {
            const double g = confirm(D, gap);
            if (g <= tol) return g;
        }
    }
    if (sv->solve_in_set.n < (size_t)sv->n) sv->solve_in_set.alloc((size_t)sv->n);
    Extracted ex;
    ex.have = true;
    double D = 0.0;
    extract_api(sv, true, sv->solve_in_set.p, &ex.num_unit, &ex.num_w, &ex.den, &D, nullptr, s,
                &ex.w_exact);
    if (!best.have || at_least_as_dense(ex, best)) {
        best = ex;
        LOWD_HIP(hipMemcpyAsync(best_in_set, sv->solve_in_set.p, (size_t)sv->n,
                                hipMemcpyDeviceToDevice, s));
    }
    return confirm(D, relative_gap(D, density_of(best)));
}

extern "C" {

lowd_status lowd_solve(lowd_solver *sv, double tol, int32_t max_sweeps, int32_t check_every,
                       uint8_t *in_set, int64_t *num_unit, double *num_w, int64_t *den,
                       double *D_out, double *gap_out, int32_t *sweeps_used, void *stream) {
    bool converged = false;
    lowd_status st = guarded([&] {
        if (!sv) fail(LOWD_E_ARG, "solver is NULL");
        if (!in_set) fail(LOWD_E_ARG, "in_set is NULL");
        if (!(tol >= 0.0)) fail(LOWD_E_ARG, "tol must be >= 0");
        if (max_sweeps < 0) fail(LOWD_E_ARG, "max_sweeps must be >= 0");
        if (check_every < 1) fail(LOWD_E_ARG, "check_every must be >= 1");
        hipStream_t s = (hipStream_t)stream;
        Extracted best;
        std::vector<std::pair<int64_t, double>> hist;
        int32_t sweeps = 0;
        double gap = 1.0e300, D = 0.0;
        // The cost of a check against a sweep's, timed with events on the
        // stream: checks without a predicted convergence point stay at
        // least k_min sweeps apart, so that they cost at most about a
        // quarter of the sweeps between them.
        hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
        struct Events {
            hipEvent_t *e;
            ~Events() {
                for (int i = 0; i < 3; ++i)
                    if (e[i]) (void)hipEventDestroy(e[i]);
            }
        } ev_guard{ev};
        for (int i = 0; i < 3; ++i) LOWD_HIP(hipEventCreate(&ev[i]));
        int32_t k_min = 1;
        while (sweeps < max_sweeps && gap > tol) {
            const int32_t k = std::min(next_check(hist, tol, check_every, k_min),
                                       max_sweeps - sweeps);
            LOWD_HIP(hipEventRecord(ev[0], s));
            if (sv->exec)
                for (int32_t t = 0; t < k; ++t) LOWD_HIP(hipGraphLaunch(sv->exec, s));
            LOWD_HIP(hipEventRecord(ev[1], s));
            sweeps += k;
            gap = certify(sv, best, in_set, tol, &D, s);
            LOWD_HIP(hipEventRecord(ev[2], s));
            hist.emplace_back(sweeps, gap);
            if (gap > tol && k > 0) {
                LOWD_HIP(hipEventSynchronize(ev[2]));
                float sweep_ms = 0.f, check_ms = 0.f;
                LOWD_HIP(hipEventElapsedTime(&sweep_ms, ev[0], ev[1]));
                LOWD_HIP(hipEventElapsedTime(&check_ms, ev[1], ev[2]));
                const double per = (double)sweep_ms / (double)k;
                k_min = per > 0.0 ? (int32_t)std::min<double>(
                                        check_every, std::max(1.0, std::ceil(4.0 * check_ms / per)))
                                  : check_every;
            }
        }
        if (!best.have) gap = certify(sv, best, in_set, tol, &D, s);   // max_sweeps == 0
        if (gap > tol && sv->state != LOWD_STATE_F64) {
            // stopped at max_sweeps: report the bound of the stored fractions
            check_impl(sv, false, &D, nullptr, nullptr, s);
            gap = relative_gap(D, density_of(best));
        }
        LOWD_HIP(hipStreamSynchronize(s));
        if (num_unit) *num_unit = sv->weighted ? 0 : best.num_unit;
        if (num_w) *num_w = best.num_w;
        if (den) *den = best.den;
        if (D_out) *D_out = D;
        if (gap_out) *gap_out = gap;
        if (sweeps_used) *sweeps_used = sweeps;
        converged = gap <= tol;
    });
    if (st == LOWD_OK && !converged) return LOWD_NOT_CONVERGED;
    return st;
}

lowd_status lowd_convergence_trace(lowd_solver *sv, int32_t sweeps, int32_t every, double *out,
                                   int64_t *points, void *stream) {
    return guarded([&] {
        if (!sv) fail(LOWD_E_ARG, "solver is NULL");
        if (sweeps < 0 || every < 1) fail(LOWD_E_ARG, "need sweeps >= 0 and every >= 1");
        if (!out || !points) fail(LOWD_E_ARG, "NULL output");
        hipStream_t s = (hipStream_t)stream;
        if (sv->ldd_in_set.n < (size_t)sv->n) sv->ldd_in_set.alloc((size_t)sv->n);
        int64_t p = 0;
        int32_t done = 0;
        for (;;) {
            double D = 0.0, rho = 0.0, gap = 0.0;
            int64_t num = 0, den = 0;
            double numw = 0.0;
            lowd_status st = lowd_extract_densest(sv, sv->ldd_in_set.p, &num, &numw, &den, &D,
                                                  &gap, stream);
            if (st != LOWD_OK) fail(st, g_last_error);
            double o[3];
            stats(sv, o, s);   // loads are current from the extraction
            rho = numw / (double)den;
            double *row = out + p * 5;
            row[0] = (double)done;
            row[1] = D;
            row[2] = rho;
            row[3] = o[2];
            row[4] = gap;
            ++p;
            if (done >= sweeps) break;
            const int32_t k = std::min(every, sweeps - done);
            if (sv->exec)
                for (int32_t t = 0; t < k; ++t) LOWD_HIP(hipGraphLaunch(sv->exec, s));
            done += k;
        }
        *points = p;
    });
}

lowd_status lowd_dks_bound(const int64_t *k_end, const double *f_end, int64_t nlevels, int64_t k,
                           double *bound) {
    return guarded([&] {
        if (!k_end || !f_end || !bound || nlevels < 1) fail(LOWD_E_ARG, "empty decomposition");
        if (k < 1 || k > k_end[nlevels - 1]) fail(LOWD_E_ARG, "k must be in [1, n]");
        int64_t kp = 0;
        double fp = 0.0;
        for (int64_t j = 0; j < nlevels; ++j) {
            if (k <= k_end[j]) {
                const double lam = (f_end[j] - fp) / (double)(k_end[j] - kp);
                *bound = (fp + (double)(k - kp) * lam) / (double)k;
                return;
            }
            kp = k_end[j];
            fp = f_end[j];
        }
    });
}

lowd_status lowd_ldd_readout(lowd_solver *sv, int32_t *level, int64_t *k_end, double *f_end,
                             int64_t *nlevels, void *stream) {
    return guarded([&] {
        if (!sv) fail(LOWD_E_ARG, "solver is NULL");
        if (!level || !k_end || !f_end || !nlevels) fail(LOWD_E_ARG, "NULL output");
        hipStream_t s = (hipStream_t)stream;
        loads_f64(sv, s);
        if (sv->ldd_in_set.n < (size_t)sv->n) sv->ldd_in_set.alloc((size_t)sv->n);
        ExtractArgs a;
        a.n = sv->n;
        a.m = sv->m;
        a.weighted = sv->weighted;
        a.L64 = sv->L64.p;
        a.row_ptr = sv->csr.row_ptr.p;
        a.inc = sv->csr.inc.p;
        a.src = sv->e_src.p;
        a.dst = sv->e_dst.p;
        a.w = sv->weighted ? sv->e_w.p : nullptr;
        a.wi = sv->weighted ? sv->e_wi.p : nullptr;
        a.wi_inc = sv->weighted ? sv->e_wi_inc.p : nullptr;
        a.wq = sv->wq;
        if (sv->m > 0) {
            a.adj = sv->adj.p;
            a.big = sv->big.p;
            a.nbig = sv->nbig;
        }
        a.in_set = sv->ldd_in_set.p;
        launch_ldd(a, sv->ex, sv->ldd, level, k_end, f_end, nlevels, s);
    });
}

lowd_status lowd_read_state(const lowd_solver *sv, double *x, double *load, void *stream) {
    return guarded([&] {
        if (!sv) fail(LOWD_E_ARG, "solver is NULL");
        hipStream_t s = (hipStream_t)stream;
        if (x && sv->m > 0) sv->fn.read_x(sv->m, sv->edge_slot.p, sv->slot_x.p, x, s);
        if (load) sv->fn.read_loads(sv->n, sv->home.p, sv->E.p, load, s);
        LOWD_HIP(hipGetLastError());
    });
}

lowd_status lowd_schedule_export(const lowd_solver *sv, int32_t *phase, int32_t *center,
                                 int32_t *nphases) {
    return guarded([&] {
        if (!sv) fail(LOWD_E_ARG, "solver is NULL");
        if (phase && sv->m > 0) memcpy(phase, sv->sch.phase.data(), (size_t)sv->m * 4);
        if (center && sv->m > 0) memcpy(center, sv->sch.center.data(), (size_t)sv->m * 4);
        if (nphases) *nphases = sv->sch.P;
    });
}

lowd_status lowd_schedule_build(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                                int32_t star_max, int32_t *phase, int32_t *center,
                                int32_t *nphases) {
    return guarded([&] {
        if (n < 1) fail(LOWD_E_ARG, "n must be >= 1");
        if (m < 0 || m >= ((int64_t)1 << 31)) fail(LOWD_E_ARG, "m must be in [0, 2^31)");
        if (m > 0 && (!src || !dst)) fail(LOWD_E_ARG, "src/dst is NULL");
        if (star_max < 1 || star_max > 254) fail(LOWD_E_ARG, "star_max must be in [1, 254]");
        for (int64_t e = 0; e < m; ++e)
            if (src[e] < 0 || src[e] >= n || dst[e] < 0 || dst[e] >= n || src[e] == dst[e])
                fail(LOWD_E_GRAPH, "invalid edge at index " + std::to_string(e));
        Schedule sc;
        build_schedule(n, m, src, dst, star_max, 0, 0, -2, -1, sc);
        if (phase && m > 0) memcpy(phase, sc.phase.data(), (size_t)m * 4);
        if (center && m > 0) memcpy(center, sc.center.data(), (size_t)m * 4);
        if (nphases) *nphases = sc.P;
    });
}

lowd_status lowd_solver_info(const lowd_solver *sv, int64_t *info) {
    return guarded([&] {
        if (!sv || !info) fail(LOWD_E_ARG, "NULL argument");
        int64_t mid_edges = 0;
        for (int32_t p = sv->sch.P1; p < sv->sch.P0; ++p) mid_edges += sv->sch.phase_edges[(size_t)p];
        info[0] = sv->n;
        info[1] = sv->m;
        info[2] = sv->sch.P;
        info[3] = sv->sch.P1;
        info[4] = sv->sch.P0 - sv->sch.P1;
        info[5] = sv->sch.P - sv->sch.P0;
        info[6] = sv->ntail;
        info[7] = sv->sch.tail_edges;
        info[8] = mid_edges;
        info[9] = sv->state;
        info[10] = sv->node_layout ? 1 : 0;
        int64_t pulled = 0;
        for (const uint8_t x : sv->sch.pull) pulled += x;
        info[11] = pulled;
    });
}

void lowd_solver_free(lowd_solver *sv) {
    if (!sv) return;
    (void)hipDeviceSynchronize();
    delete sv;
}

lowd_status lowd_prune(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                       uint8_t *node_keep, int32_t *relabel, int32_t *h_src, int32_t *h_dst,
                       int64_t *edge_map, int32_t *rounds, int32_t *n_h, int64_t *m_h,
                       void *stream) {
    return guarded([&] {
        if (n < 1) fail(LOWD_E_ARG, "n must be >= 1");
        if (m < 0 || m >= ((int64_t)1 << 31)) fail(LOWD_E_ARG, "m must be in [0, 2^31)");
        if (m > 0 && (!src || !dst)) fail(LOWD_E_ARG, "src/dst is NULL");
        if (!node_keep) fail(LOWD_E_ARG, "node_keep is NULL");
        if ((h_src == nullptr) != (h_dst == nullptr)) fail(LOWD_E_ARG, "h_src/h_dst: both or none");
        hipStream_t s = (hipStream_t)stream;
        // one allocation serves the check and then the prune
        const size_t need = std::max(validate_ws_bytes(n, m, nullptr),
                                     prune_ws_bytes(n, m, h_src != nullptr, edge_map != nullptr));
        DBuf<char> buf(need);
        Arena ws(buf.p, buf.bytes());
        validate_graph_ws(n, m, src, dst, nullptr, ws, s);
        PruneResult r =
            run_prune_ws(n, m, src, dst, node_keep, relabel, h_src, h_dst, edge_map, ws, s);
        if (rounds) *rounds = r.rounds;
        if (n_h) *n_h = r.n_h;
        if (m_h) *m_h = r.m_h;
    });
}

}  // extern "C"

// ------------------------------------------------- allocation-free prune --
// lowd_prune_noalloc takes every device buffer from this file-scope array.
// Each GPU the library runs on holds its own copy until the process ends.
// Host code reaches a device's copy only through the address
// hipGetSymbolAddress returns on that device, taken once per device.
constexpr size_t kNoAllocScratchBytes = (size_t)128 << 20;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

void *scratch_on_current_device() {
    int dev = 0;
    LOWD_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) fail(LOWD_E_UNSUPPORTED, "device index beyond 63");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        LOWD_HIP(hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = ptr;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" {

lowd_status lowd_prune_noalloc(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                               uint8_t *node_keep, int32_t *relabel, int32_t *h_src,
                               int32_t *h_dst, int64_t *edge_map, int32_t *rounds, int32_t *n_h,
                               int64_t *m_h, void *stream) {
    return guarded([&] {
        if (n < 1) fail(LOWD_E_ARG, "n must be >= 1");
        if (m < 0 || m >= ((int64_t)1 << 31)) fail(LOWD_E_ARG, "m must be in [0, 2^31)");
        if (m > 0 && (!src || !dst)) fail(LOWD_E_ARG, "src/dst is NULL");
        if (!node_keep) fail(LOWD_E_ARG, "node_keep is NULL");
        if ((h_src == nullptr) != (h_dst == nullptr)) fail(LOWD_E_ARG, "h_src/h_dst: both or none");
        const size_t need = std::max(validate_ws_bytes(n, m, nullptr),
                                     prune_ws_bytes(n, m, h_src != nullptr, edge_map != nullptr));
        if (need > kNoAllocScratchBytes)
            fail(LOWD_E_UNSUPPORTED, "this graph needs " + std::to_string(need) +
                                         " bytes of scratch; lowd_prune_noalloc holds " +
                                         std::to_string(kNoAllocScratchBytes));
        hipStream_t s = (hipStream_t)stream;
        Arena ws(scratch_on_current_device(), kNoAllocScratchBytes);
        validate_graph_ws(n, m, src, dst, nullptr, ws, s);
        PruneResult r =
            run_prune_ws(n, m, src, dst, node_keep, relabel, h_src, h_dst, edge_map, ws, s);
        if (rounds) *rounds = r.rounds;
        if (n_h) *n_h = r.n_h;
        if (m_h) *m_h = r.m_h;
    });
}

lowd_status lowd_prune_weighted(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                                const float *w, uint8_t *node_keep, int32_t *relabel,
                                int32_t *h_src, int32_t *h_dst, float *h_w, int64_t *edge_map,
                                int32_t *rounds, int32_t *n_h, int64_t *m_h, double *w_h,
                                void *stream) {
    return guarded([&] {
        if (n < 1) fail(LOWD_E_ARG, "n must be >= 1");
        if (m < 0 || m >= ((int64_t)1 << 31)) fail(LOWD_E_ARG, "m must be in [0, 2^31)");
        if (m > 0 && (!src || !dst || !w)) fail(LOWD_E_ARG, "src/dst/w is NULL");
        if (!node_keep) fail(LOWD_E_ARG, "node_keep is NULL");
        if ((h_src == nullptr) != (h_dst == nullptr)) fail(LOWD_E_ARG, "h_src/h_dst: both or none");
        hipStream_t s = (hipStream_t)stream;
        validate_graph(n, m, src, dst, w, s);
        PruneResult r = run_prune_weighted(n, m, src, dst, w, node_keep, relabel, h_src, h_dst,
                                           h_w, edge_map, w_h, s);
        if (rounds) *rounds = r.rounds;
        if (n_h) *n_h = r.n_h;
        if (m_h) *m_h = r.m_h;
    });
}

lowd_status lowd_greedy_peel(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                             int32_t *order, int64_t *rem_m, uint8_t *in_set, int64_t *num,
                             int64_t *den, void *stream) {
    return guarded([&] {
        if (n < 1) fail(LOWD_E_ARG, "n must be >= 1");
        if (m < 0 || m >= ((int64_t)1 << 31)) fail(LOWD_E_ARG, "m must be in [0, 2^31)");
        if (m > 0 && (!src || !dst)) fail(LOWD_E_ARG, "src/dst is NULL");
        if (!order || !rem_m) fail(LOWD_E_ARG, "order/rem_m is NULL");
        hipStream_t s = (hipStream_t)stream;
        validate_graph(n, m, src, dst, nullptr, s);
        const int64_t bi = greedy_peel(n, m, src, dst, order, rem_m, in_set,
                                       (int64_t)32 << 30, s);
        int64_t mm = m;
        if (bi > 0) {
            LOWD_HIP(hipMemcpyAsync(&mm, rem_m + (bi - 1), sizeof(mm), hipMemcpyDeviceToHost, s));
            LOWD_HIP(hipStreamSynchronize(s));
        }
        if (num) *num = mm;
        if (den) *den = (int64_t)n - bi;
    });
}

}  // extern "C"

// ---------------------------------------------------------------- batches --
struct lowd_batch {
    int32_t G = 0;
    int64_t N = 0, M = 0;
    int32_t state = 0;
    SweepLaunch fn{};
    std::vector<int64_t> node_ptr_h, edge_ptr_h;
    int64_t max_nodes = 0;   // nodes of the largest graph
    int64_t total_phases = 0, max_phases = 0;
    DBuf<int64_t> node_ptr, edge_ptr, desc_ptr, slot_edge;
    DBuf<int32_t> gsrc, gdst, node_graph, order_all, order, active, tile_center, deg;
    DBuf<int64_t> active_edges;
    DBuf<PhaseDesc> descs;
    DBuf<uint32_t> slot_leaf;
    DBuf<char> slot_x, Lstate;
    DBuf<double> L64;
    DBuf<unsigned> queue;
    // FP32K: the incidence of the concatenated graphs and each edge's slot,
    // to recompute FP64 loads from the fractions (the dual bound must be the
    // loads of the stored fractions)
    Csr csr;
    DBuf<int64_t> edge_slot;
    DBuf<uint8_t> active_flag;   // [G]
    // the graphs still iterating as the host last saw them (after a reset or
    // a retire): count, each graph's index in that list (-1 if retired) and
    // the compact node offsets of the listed graphs, for the extraction
    std::vector<int32_t> order_all_h;
    int32_t act_count = 0;
    int64_t act_nodes = 0;
    std::vector<int32_t> rank_h;
    std::vector<int64_t> seg_h;
    DBuf<int32_t> act_rank;
    DBuf<int64_t> act_seg;
    // every graph's latest extraction (retired graphs keep theirs)
    DBuf<int64_t> r_num, r_den;
    DBuf<double> r_D;
    DBuf<uint8_t> r_in_set;
    BatchExtractScratch ex;
    size_t lds = 0;        // bytes of LDS per workgroup
    int32_t waves = 8;     // launch shape: waves per workgroup,
    int32_t prefetch = 1;  // double-buffered tiles or not,
    int32_t blocks = 1;    // workgroups
    int32_t shape() const { return waves * 2 + prefetch; }
    // Once few graphs still iterate, each runs alone on a CU and its widest
    // phases (more tiles than waves) bound the launch: then 16 waves per
    // workgroup (no tile prefetch, to stay within 128 registers) deal those
    // tiles out faster.  FP32K only (the FP64 kernel would spill at 16
    // waves); off when the shape is forced.
    bool tail_shape = false;
    int32_t cus = 1;
    int32_t last_active = 0;   // graphs iterating after the last retire
    static constexpr int32_t kTailShape = 16 * 2 + 0;
    int32_t graph_sweeps = -1, graph_shape = -1;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t per_cu = 1;   // workgroups per CU of the tuned shape
    // the batched solve in one launch: the batch's adjacency (the other end
    // of each incidence entry), per-node scratch of the in-kernel checks,
    // the per-graph sweep counts, and the captured launch with its settings
    DBuf<int32_t> adj;
    DBuf<uint32_t> inc_slot;   // FP32K: slot << 1 | side of each incidence entry
    DBuf<uint64_t> sk0, sk1;
    DBuf<uint32_t> si0, si1;
    DBuf<int32_t> spos, shist, r_sweeps, r_set;
    hipGraph_t solve_graph = nullptr;
    hipGraphExec_t solve_exec = nullptr;
    int32_t solve_shape = -1, solve_blocks = -1, solve_max = -1, solve_every = -1;
    double solve_tol = -1.0;
    void drop_solve_graph() {
        if (solve_exec) (void)hipGraphExecDestroy(solve_exec);
        if (solve_graph) (void)hipGraphDestroy(solve_graph);
        solve_exec = nullptr;
        solve_graph = nullptr;
        solve_shape = -1;
    }
    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
        graph_sweeps = -1;
        graph_shape = -1;
    }
    ~lowd_batch() {
        drop_graph();
        drop_solve_graph();
    }
};

// The extraction's view of the graphs still iterating: act[0..A) as listed
// on the device (b->order), their ranks and compact node offsets.
static void set_active_list(lowd_batch *b, const int32_t *act, int32_t A, hipStream_t s) {
    b->rank_h.assign((size_t)b->G, -1);
    b->seg_h.assign((size_t)A + 1, 0);
    for (int32_t k = 0; k < A; ++k) {
        const int32_t g = act[k];
        b->rank_h[(size_t)g] = k;
        b->seg_h[(size_t)k + 1] = b->seg_h[(size_t)k] + (b->node_ptr_h[(size_t)g + 1] -
                                                         b->node_ptr_h[(size_t)g]);
    }
    b->act_count = A;
    b->act_nodes = b->seg_h[(size_t)A];
    LOWD_HIP(hipMemcpyAsync(b->act_rank.p, b->rank_h.data(), b->rank_h.size() * sizeof(int32_t),
                            hipMemcpyHostToDevice, s));
    LOWD_HIP(hipMemcpyAsync(b->act_seg.p, b->seg_h.data(), b->seg_h.size() * sizeof(int64_t),
                            hipMemcpyHostToDevice, s));
    // the host vectors may change at the next reset or retire: let the
    // copies finish first
    LOWD_HIP(hipStreamSynchronize(s));
}

static void batch_reset(lowd_batch *b, hipStream_t s) {
    const int64_t nslots = (int64_t)(b->slot_leaf.n);
    if (b->M > 0) b->fn.init_slots(nslots, b->slot_edge.p, nullptr, b->slot_x.p, nullptr, s);
    b->fn.batch_init_loads(b->N, b->deg.p, b->Lstate.p, s);
    launch_activate_all(b->G, b->order_all.p, b->edge_ptr.p, b->order.p, b->active.p,
                        b->active_edges.p, s);
    LOWD_HIP(hipGetLastError());
    b->last_active = b->G;
    set_active_list(b, b->order_all_h.data(), b->G, s);
}

// One launch of the persistent kernel for `sweeps` sweeps, as a HIP graph
// (captured once per distinct sweep count and launch shape).
static void batch_launch(lowd_batch *b, int32_t sweeps, hipStream_t s) {
    int32_t shape = b->shape(), blocks = b->blocks;
    if (b->tail_shape && b->last_active <= 2 * b->cus) {
        shape = lowd_batch::kTailShape;
        blocks = std::min(b->cus, b->G);
    }
    if (b->graph_sweeps != sweeps || b->graph_shape != shape || !b->exec) {
        b->drop_graph();
        hipStream_t cs;
        LOWD_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        hipError_t err = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (err == hipSuccess) {
            b->fn.batch(shape, b->active.p, b->order.p, b->queue.p, b->node_ptr.p, b->desc_ptr.p,
                        b->descs.p, b->tile_center.p, b->slot_leaf.p, b->slot_x.p, sweeps,
                        b->Lstate.p, b->lds, blocks, cs);
            err = hipStreamEndCapture(cs, &b->graph);
        }
        (void)hipStreamDestroy(cs);
        LOWD_HIP(err);
        LOWD_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
        b->graph_sweeps = sweeps;
        b->graph_shape = shape;
    }
    LOWD_HIP(hipGraphLaunch(b->exec, s));
}

// Launch-shape autotuner: every shape (waves per workgroup x workgroups per
// CU) runs a short stretch of the real batch, timed with events; the
// fastest is kept and the state is reset.  The shape changes only which
// workgroup runs which graph and how a graph's tiles are dealt to its waves,
// never the result.
static void batch_tune(lowd_batch *b, int32_t cus, hipStream_t s) {
    struct Shape { int32_t waves, prefetch, per_cu; };
    const Shape shapes[] = {{8, 1, 1}, {8, 0, 1}, {8, 0, 2}, {4, 1, 1}, {4, 1, 2},
                            {4, 0, 2}, {4, 0, 3}, {4, 0, 4}};
    hipEvent_t e0, e1;
    LOWD_HIP(hipEventCreate(&e0));
    LOWD_HIP(hipEventCreate(&e1));
    float best = 1e30f;
    Shape pick{b->waves, b->prefetch, 1};
    const int32_t tune_sweeps = 2;
    for (const Shape &sh : shapes) {
        if ((int64_t)b->lds * sh.per_cu > 160 * 1024) continue;
        b->waves = sh.waves;
        b->prefetch = sh.prefetch;
        b->blocks = (int32_t)std::min<int64_t>((int64_t)cus * sh.per_cu, b->G);
        b->drop_graph();
        b->fn.set_batch_lds(b->shape(), b->lds);
        batch_reset(b, s);
        batch_launch(b, tune_sweeps, s);   // first launch: instantiation, cold caches
        LOWD_HIP(hipEventRecord(e0, s));
        batch_launch(b, tune_sweeps, s);
        LOWD_HIP(hipEventRecord(e1, s));
        LOWD_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        LOWD_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (ms < best) {
            best = ms;
            pick = sh;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    b->waves = pick.waves;
    b->prefetch = pick.prefetch;
    b->blocks = (int32_t)std::min<int64_t>((int64_t)cus * pick.per_cu, b->G);
    b->per_cu = pick.per_cu;
    b->drop_graph();
    b->fn.set_batch_lds(b->shape(), b->lds);
}

extern "C" {

lowd_status lowd_batch_prepare(int32_t G, const int64_t *node_ptr, const int64_t *edge_ptr,
                               const int32_t *src, const int32_t *dst, int32_t state,
                               int32_t star_max, int32_t tune, lowd_batch **out, void *stream) {
    return guarded([&] {
        if (!out) fail(LOWD_E_ARG, "out is NULL");
        *out = nullptr;
        if (G < 1 || !node_ptr || !edge_ptr) fail(LOWD_E_ARG, "G >= 1 and node_ptr/edge_ptr needed");
        if (state != LOWD_STATE_F64 && state != LOWD_STATE_F32K) fail(LOWD_E_ARG, "bad state");
        if (star_max < 1 || star_max > kTierStar) fail(LOWD_E_ARG, "star_max must be in [1, 16]");
        if (tune != 0 && tune != 1) fail(LOWD_E_ARG, "tune must be 0 or 1");
        if (node_ptr[0] != 0 || edge_ptr[0] != 0) fail(LOWD_E_ARG, "node_ptr[0], edge_ptr[0] must be 0");
        for (int32_t g = 0; g < G; ++g) {
            if (node_ptr[g + 1] - node_ptr[g] < 1) fail(LOWD_E_ARG, "every graph needs a node");
            if (edge_ptr[g + 1] < edge_ptr[g]) fail(LOWD_E_ARG, "edge_ptr must not decrease");
        }
        const int64_t N = node_ptr[G], M = edge_ptr[G];
        if (N > 0x7FFFFFFD || M >= ((int64_t)1 << 31)) fail(LOWD_E_ARG, "batch too large");
        if (M > 0 && (!src || !dst)) fail(LOWD_E_ARG, "src/dst is NULL");
        hipStream_t s = (hipStream_t)stream;
        auto b = new lowd_batch();
        std::unique_ptr<lowd_batch> guard(b);
        b->G = G;
        b->N = N;
        b->M = M;
        b->state = state;
        get_sweep_launchers(state, false, b->fn);
        b->node_ptr_h.assign(node_ptr, node_ptr + G + 1);
        b->edge_ptr_h.assign(edge_ptr, edge_ptr + G + 1);
        for (int32_t g = 0; g < G; ++g)
            b->max_nodes = std::max<int64_t>(b->max_nodes, node_ptr[g + 1] - node_ptr[g]);

        std::vector<int32_t> hs((size_t)M), hd((size_t)M);
        if (M > 0) {
            LOWD_HIP(hipMemcpyAsync(hs.data(), src, (size_t)M * 4, hipMemcpyDeviceToHost, s));
            LOWD_HIP(hipMemcpyAsync(hd.data(), dst, (size_t)M * 4, hipMemcpyDeviceToHost, s));
            LOWD_HIP(hipStreamSynchronize(s));
        }
        std::vector<int32_t> gsrc((size_t)M), gdst((size_t)M), node_graph((size_t)N);
        for (int32_t g = 0; g < G; ++g) {
            const int64_t ng = node_ptr[g + 1] - node_ptr[g];
            for (int64_t u = node_ptr[g]; u < node_ptr[g + 1]; ++u) node_graph[(size_t)u] = g;
            for (int64_t e = edge_ptr[g]; e < edge_ptr[g + 1]; ++e) {
                const int32_t a = hs[(size_t)e], c = hd[(size_t)e];
                if (a < 0 || a >= ng || c < 0 || c >= ng || a == c)
                    fail(LOWD_E_GRAPH, "invalid edge " + std::to_string(e) + " of graph " +
                                           std::to_string(g) + ": (" + std::to_string(a) + ", " +
                                           std::to_string(c) + "), n = " + std::to_string(ng));
                gsrc[(size_t)e] = a + (int32_t)node_ptr[g];
                gdst[(size_t)e] = c + (int32_t)node_ptr[g];
            }
        }
        upload(b->gsrc, gsrc, s);
        upload(b->gdst, gdst, s);
        upload(b->node_graph, node_graph, s);
        {
            int64_t bad = find_duplicate_pair((int32_t)N, M, b->gsrc.p, b->gdst.p, s);
            if (bad >= 0) fail(LOWD_E_GRAPH, "repeated pair at edge " + std::to_string(bad));
        }

        // per-graph schedules (every phase from LDS), built in parallel
        const int64_t lds_cap = (int64_t)lds_capacity_bytes() - (int64_t)kWgCheckLdsMax;
        std::vector<Schedule> sch((size_t)G);
        {
            std::atomic<int32_t> next(0);
            std::atomic<int32_t> bad(-1);
            unsigned nt = std::thread::hardware_concurrency();
            if (nt < 1) nt = 1;
            if (nt > 16) nt = 16;
            std::vector<std::thread> pool;
            std::vector<std::string> errs(nt);
            for (unsigned t = 0; t < nt; ++t)
                pool.emplace_back([&, t] {
                    try {
                        for (int32_t g = next++; g < G; g = next++) {
                            const int64_t e0 = edge_ptr[g];
                            build_schedule((int32_t)(node_ptr[g + 1] - node_ptr[g]),
                                           edge_ptr[g + 1] - e0, hs.data() + e0, hd.data() + e0,
                                           star_max, lds_cap, (int64_t)b->fn.l_bytes, 0, 0,
                                           sch[(size_t)g], true);
                        }
                    } catch (const Error &e) {
                        errs[t] = e.msg;
                        bad = 1;
                    } catch (...) {
                        errs[t] = "schedule failed";
                        bad = 1;
                    }
                });
            for (auto &th : pool) th.join();
            if (bad >= 0)
                for (auto &e : errs)
                    if (!e.empty()) fail(LOWD_E_ARG, e);
        }
        // concatenate the layouts; every graph must fit one workgroup's LDS
        std::vector<PhaseDesc> descs;
        std::vector<int32_t> tile_center;
        std::vector<uint32_t> slot_leaf;
        std::vector<int64_t> slot_edge, desc_ptr((size_t)G + 1, 0);
        const bool recompute = state == LOWD_STATE_F32K && M > 0;
        std::vector<int64_t> edge_slot(recompute ? (size_t)M : 0);
        size_t lds_need = 0;
        for (int32_t g = 0; g < G; ++g) {
            const Schedule &sc = sch[(size_t)g];
            const int64_t ng = node_ptr[g + 1] - node_ptr[g];
            const size_t need = tail_desc_bytes(sc.P) + (size_t)(ng + 2) * b->fn.l_bytes;
            if ((int64_t)need > lds_cap)
                fail(LOWD_E_UNSUPPORTED, "graph " + std::to_string(g) + " (" + std::to_string(ng) +
                                             " nodes, " + std::to_string(sc.P) +
                                             " phases) does not fit one workgroup's LDS");
            if (need > lds_need) lds_need = need;
            b->total_phases += sc.P;
            b->max_phases = std::max<int64_t>(b->max_phases, sc.P);
            const int64_t slot0 = (int64_t)slot_leaf.size();
            const int32_t tile0 = (int32_t)(tile_center.size() / kWave);
            for (const PhaseDescWide &dw : sc.desc) {
                PhaseDesc d = narrow_desc<kTierStar>(dw);
                d.slot_base += slot0;
                d.tile0 += tile0;
                descs.push_back(d);
            }
            desc_ptr[(size_t)g + 1] = (int64_t)descs.size();
            tile_center.insert(tile_center.end(), sc.tile_center.begin(), sc.tile_center.end());
            slot_leaf.insert(slot_leaf.end(), sc.slot_leaf.begin(), sc.slot_leaf.end());
            for (int64_t e : sc.slot_edge) slot_edge.push_back(e >= 0 ? e + edge_ptr[g] : -1);
            if (recompute)
                for (size_t e = 0; e < sc.edge_slot.size(); ++e)
                    edge_slot[(size_t)edge_ptr[g] + e] = slot0 + sc.edge_slot[e];
        }
        // the incidence of the concatenated graphs and the other end of each
        // entry: the in-kernel checks count each node's neighbours at higher
        // positions, and FP32K recomputes the fractions' loads along it
        build_incidence((int32_t)N, M, b->gsrc.p, b->gdst.p, b->csr, s);
        b->adj.alloc((size_t)(2 * M > 0 ? 2 * M : 1));
        if (M > 0) build_adjacency(M, b->csr, b->gsrc.p, b->gdst.p, b->adj.p, s);
        if (recompute) {
            upload(b->edge_slot, edge_slot, s);
            b->active_flag.alloc((size_t)G);
            b->inc_slot.alloc((size_t)(2 * M));
            launch_inc_slots(2 * M, b->csr.inc.p, b->edge_slot.p, b->inc_slot.p, s);
        }
        std::vector<int32_t> order((size_t)G);
        for (int32_t g = 0; g < G; ++g) order[(size_t)g] = g;
        std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t c) {
            return edge_ptr[a + 1] - edge_ptr[a] > edge_ptr[c + 1] - edge_ptr[c];
        });
        upload(b->node_ptr, b->node_ptr_h, s);
        upload(b->edge_ptr, b->edge_ptr_h, s);
        upload(b->desc_ptr, desc_ptr, s);
        upload(b->slot_edge, slot_edge, s);
        upload(b->order_all, order, s);
        b->order_all_h = order;
        b->act_rank.alloc((size_t)G);
        b->act_seg.alloc((size_t)G + 1);
        b->r_num.alloc((size_t)G);
        b->r_den.alloc((size_t)G);
        b->r_D.alloc((size_t)G);
        b->r_in_set.alloc((size_t)N);
        LOWD_HIP(hipMemsetAsync(b->r_num.p, 0, b->r_num.bytes(), s));
        LOWD_HIP(hipMemsetAsync(b->r_den.p, 0, b->r_den.bytes(), s));
        LOWD_HIP(hipMemsetAsync(b->r_D.p, 0, b->r_D.bytes(), s));
        LOWD_HIP(hipMemsetAsync(b->r_in_set.p, 0, b->r_in_set.bytes(), s));
        b->order.alloc((size_t)G);
        b->active.alloc(1);
        b->active_edges.alloc(1);
        upload(b->tile_center, tile_center, s);
        upload(b->descs, descs, s);
        upload(b->slot_leaf, slot_leaf, s);
        const int64_t nslots = (int64_t)slot_leaf.size();
        b->slot_x.alloc((size_t)(nslots > 0 ? nslots : 1) * b->fn.x_bytes);
        b->Lstate.alloc((size_t)(N > 0 ? N : 1) * b->fn.l_bytes);
        b->L64.alloc((size_t)(N > 0 ? N : 1));
        b->deg.alloc((size_t)(N > 0 ? N : 1));
        launch_batch_degrees(N, M, b->gsrc.p, b->gdst.p, b->deg.p, s);
        b->queue.alloc(2);
        b->lds = lds_need;

        int dev = 0, cus = 0;
        LOWD_HIP(hipGetDevice(&dev));
        LOWD_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        b->waves = 8;
        b->prefetch = 1;
        int32_t per_cu = 1;
        if (const char *e = getenv("LOWD_BATCH_SHAPE")) {   // "waves,prefetch,per_cu"
            int w = 0, pf = 0, pc = 0;
            if (sscanf(e, "%d,%d,%d", &w, &pf, &pc) != 3 || (w != 4 && w != 8 && w != 16) ||
                (pf != 0 && pf != 1) || (w == 16 && pf != 0) || pc < 1 || pc > 4)
                fail(LOWD_E_ARG, "LOWD_BATCH_SHAPE must be waves(4|8),prefetch(0|1),per_cu(1-4) "
                                 "or 16,0,per_cu");
            b->waves = w;
            b->prefetch = pf;
            per_cu = pc;
        }
        b->blocks = (int32_t)std::min<int64_t>((int64_t)cus * per_cu, G);
        b->per_cu = per_cu;
        b->cus = cus;
        b->fn.set_batch_lds(b->shape(), b->lds);
        if (tune) batch_tune(b, cus, s);
        if (state == LOWD_STATE_F32K && !getenv("LOWD_BATCH_SHAPE")) {
            b->fn.set_batch_lds(lowd_batch::kTailShape, b->lds);
            b->tail_shape = true;
        }
        batch_reset(b, s);
        LOWD_HIP(hipStreamSynchronize(s));
        *out = guard.release();
    });
}

lowd_status lowd_batch_reset(lowd_batch *b, void *stream) {
    return guarded([&] {
        if (!b) fail(LOWD_E_ARG, "batch is NULL");
        batch_reset(b, (hipStream_t)stream);
    });
}

lowd_status lowd_batch_iterate(lowd_batch *b, int32_t sweeps, void *stream) {
    return guarded([&] {
        if (!b) fail(LOWD_E_ARG, "batch is NULL");
        if (sweeps < 0) fail(LOWD_E_ARG, "sweeps must be >= 0");
        if (sweeps == 0) return;
        batch_launch(b, sweeps, (hipStream_t)stream);
    });
}

lowd_status lowd_batch_extract(lowd_batch *b, uint8_t *in_set, int64_t *num, int64_t *den,
                               double *D, double *load, void *stream) {
    return guarded([&] {
        if (!b) fail(LOWD_E_ARG, "batch is NULL");
        if (!in_set || !num || !den) fail(LOWD_E_ARG, "in_set/num/den is NULL");
        hipStream_t s = (hipStream_t)stream;
        if (b->state == LOWD_STATE_F32K && b->M > 0) {
            // FP64 loads of the stored fractions of the graphs still
            // iterating; the carried loads restart from them, so the rounding
            // of the fractions cannot make the two drift apart for more than
            // one check interval
            b->fn.batch_recompute(b->G, b->N, b->active.p, b->order.p, b->node_graph.p,
                                  b->active_flag.p, b->csr.row_ptr.p, b->csr.inc.p,
                                  b->edge_slot.p, b->slot_x.p, b->L64.p, b->Lstate.p, s);
        } else
            b->fn.batch_loads_f64(b->N, b->Lstate.p, b->L64.p, s);
        BatchExtractArgs a;
        a.G = b->G;
        a.N = b->N;
        a.M = b->M;
        a.node_ptr = b->node_ptr.p;
        a.edge_ptr = b->edge_ptr.p;
        a.max_nodes = b->max_nodes;
        a.node_graph = b->node_graph.p;
        a.gsrc = b->gsrc.p;
        a.gdst = b->gdst.p;
        a.L64 = b->L64.p;
        a.A = b->act_count;
        a.act = b->order.p;
        a.seg = b->act_seg.p;
        a.rank = b->act_rank.p;
        a.Na = b->act_nodes;
        a.in_set = b->r_in_set.p;
        a.num = b->r_num.p;
        a.den = b->r_den.p;
        a.D = b->r_D.p;
        launch_extract_batch(a, b->ex, s);
        const size_t gb = (size_t)b->G * 8;
        LOWD_HIP(hipMemcpyAsync(num, b->r_num.p, gb, hipMemcpyDeviceToDevice, s));
        LOWD_HIP(hipMemcpyAsync(den, b->r_den.p, gb, hipMemcpyDeviceToDevice, s));
        if (D) LOWD_HIP(hipMemcpyAsync(D, b->r_D.p, gb, hipMemcpyDeviceToDevice, s));
        LOWD_HIP(hipMemcpyAsync(in_set, b->r_in_set.p, (size_t)b->N, hipMemcpyDeviceToDevice, s));
        if (load)
            LOWD_HIP(hipMemcpyAsync(load, b->L64.p, (size_t)b->N * sizeof(double),
                                    hipMemcpyDeviceToDevice, s));
    });
}

lowd_status lowd_batch_retire(lowd_batch *b, const int64_t *num, const int64_t *den,
                              const double *D, double tol, int32_t *active, int64_t *active_edges,
                              void *stream) {
    return guarded([&] {
        if (!b) fail(LOWD_E_ARG, "batch is NULL");
        if (!num || !den || !D) fail(LOWD_E_ARG, "num/den/D is NULL");
        if (!(tol >= 0.0)) fail(LOWD_E_ARG, "tol must be >= 0");
        hipStream_t s = (hipStream_t)stream;
        launch_retire(b->G, b->order_all.p, b->edge_ptr.p, num, den, D, tol, b->order.p,
                      b->active.p, b->active_edges.p, s);
        LOWD_HIP(hipGetLastError());
        int32_t a = 0;
        int64_t ae = 0;
        LOWD_HIP(hipMemcpyAsync(&a, b->active.p, sizeof(a), hipMemcpyDeviceToHost, s));
        LOWD_HIP(hipMemcpyAsync(&ae, b->active_edges.p, sizeof(ae), hipMemcpyDeviceToHost, s));
        LOWD_HIP(hipStreamSynchronize(s));
        if (active) *active = a;
        if (active_edges) *active_edges = ae;
        b->last_active = a;
        std::vector<int32_t> act((size_t)a);
        if (a > 0) {
            LOWD_HIP(hipMemcpyAsync(act.data(), b->order.p, (size_t)a * sizeof(int32_t),
                                    hipMemcpyDeviceToHost, s));
            LOWD_HIP(hipStreamSynchronize(s));
        }
        set_active_list(b, act.data(), a, s);
    });
}

lowd_status lowd_batch_info(const lowd_batch *b, int64_t *info) {
    return guarded([&] {
        if (!b || !info) fail(LOWD_E_ARG, "NULL argument");
        info[0] = b->G;
        info[1] = b->N;
        info[2] = b->M;
        info[3] = b->total_phases;
        info[4] = b->max_phases;
        info[5] = b->waves;
        info[6] = b->prefetch;
        info[7] = b->blocks;
        info[8] = (int64_t)b->lds;
    });
}

void lowd_batch_free(lowd_batch *b) {
    if (!b) return;
    (void)hipDeviceSynchronize();
    delete b;
}

// Solve to a tolerance, from the batch's current state, in one persistent
// launch (k_batch_solve, captured as a HIP graph once per launch settings):
// every graph still listed as iterating is swept and checked inside its
// workgroup until its own certified gap is within tol or max_sweeps.
lowd_status lowd_batch_solve_prepared(lowd_batch *b, double tol, int32_t max_sweeps,
                                      int32_t check_every, uint8_t *in_set, int64_t *num,
                                      int64_t *den, double *D, int32_t *sweeps_used,
                                      int32_t *set_sweeps, void *stream) {
    unsigned unconverged = 0;
    lowd_status st = guarded([&] {
        if (!b) fail(LOWD_E_ARG, "batch is NULL");
        if (!in_set || !num || !den) fail(LOWD_E_ARG, "in_set/num/den is NULL");
        if (!(tol >= 0.0)) fail(LOWD_E_ARG, "tol must be >= 0");
        if (max_sweeps < 0) fail(LOWD_E_ARG, "max_sweeps must be >= 0");
        if (check_every < 1) fail(LOWD_E_ARG, "check_every must be >= 1");
        hipStream_t s = (hipStream_t)stream;
        const size_t N = (size_t)(b->N > 0 ? b->N : 1);
        if (b->sk0.n < N) {
            b->sk0.alloc(N);
            b->sk1.alloc(N);
            b->si0.alloc(N);
            b->si1.alloc(N);
            b->spos.alloc(N);
            b->shist.alloc(N);
            b->r_sweeps.alloc((size_t)b->G);
            b->r_set.alloc((size_t)b->G);
        }
        // the tuned shape, where its sweeps and checks fit the registers
        // together without spilling (4 waves, or 8 without the prefetching
        // tile buffer); else 8 waves without it
        const int32_t shape = b->waves == 4 ? b->shape() : 8 * 2 + 0;
        // workgroups: the tuned count per CU, as far as the checks' static LDS
        // leaves room
        const int64_t per_wg = (int64_t)b->lds + (int64_t)kWgCheckLdsMax;
        const int32_t fit = (int32_t)std::max<int64_t>(1, (160 * 1024) / per_wg);
        const int32_t blocks =
            (int32_t)std::min<int64_t>((int64_t)b->cus * std::min(b->per_cu, fit), b->G);
        if (!b->solve_exec || b->solve_shape != shape || b->solve_blocks != blocks ||
            b->solve_tol != tol || b->solve_max != max_sweeps || b->solve_every != check_every) {
            b->drop_solve_graph();
            b->fn.set_batch_solve_lds(shape, b->lds);
            BatchSolveArgs a;
            a.active = b->active.p;
            a.order = b->order.p;
            a.queue = b->queue.p;
            a.node_ptr = b->node_ptr.p;
            a.desc_ptr = b->desc_ptr.p;
            a.descs = b->descs.p;
            a.tile_center = b->tile_center.p;
            a.slot_leaf = b->slot_leaf.p;
            a.slot_x = b->slot_x.p;
            a.Lstate = b->Lstate.p;
            a.row_ptr = b->csr.row_ptr.p;
            a.adj = b->adj.p;
            a.inc_slot = b->inc_slot.p;
            a.k0 = b->sk0.p;
            a.k1 = b->sk1.p;
            a.i0 = b->si0.p;
            a.i1 = b->si1.p;
            a.pos = b->spos.p;
            a.hist = b->shist.p;
            a.tol = tol;
            a.max_sweeps = max_sweeps;
            a.check_every = check_every;
            a.in_set = b->r_in_set.p;
            a.num = b->r_num.p;
            a.den = b->r_den.p;
            a.D = b->r_D.p;
            a.sweeps_used = b->r_sweeps.p;
            a.set_sweeps = b->r_set.p;
            hipStream_t cs;
            LOWD_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            hipError_t err = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (err == hipSuccess) {
                b->fn.batch_solve(shape, a, b->lds, blocks, cs);
                err = hipStreamEndCapture(cs, &b->solve_graph);
            }
            (void)hipStreamDestroy(cs);
            LOWD_HIP(err);
            LOWD_HIP(hipGraphInstantiate(&b->solve_exec, b->solve_graph, nullptr, nullptr, 0));
            b->solve_shape = shape;
            b->solve_blocks = blocks;
            b->solve_tol = tol;
            b->solve_max = max_sweeps;
            b->solve_every = check_every;
        }
        LOWD_HIP(hipGraphLaunch(b->solve_exec, s));
        const size_t gb = (size_t)b->G * 8, g4 = (size_t)b->G * 4;
        LOWD_HIP(hipMemcpyAsync(num, b->r_num.p, gb, hipMemcpyDeviceToDevice, s));
        LOWD_HIP(hipMemcpyAsync(den, b->r_den.p, gb, hipMemcpyDeviceToDevice, s));
        if (D) LOWD_HIP(hipMemcpyAsync(D, b->r_D.p, gb, hipMemcpyDeviceToDevice, s));
        LOWD_HIP(hipMemcpyAsync(in_set, b->r_in_set.p, (size_t)b->N, hipMemcpyDeviceToDevice, s));
        if (sweeps_used)
            LOWD_HIP(hipMemcpyAsync(sweeps_used, b->r_sweeps.p, g4, hipMemcpyDeviceToDevice, s));
        if (set_sweeps)
            LOWD_HIP(hipMemcpyAsync(set_sweeps, b->r_set.p, g4, hipMemcpyDeviceToDevice, s));
        LOWD_HIP(hipMemcpyAsync(&unconverged, b->queue.p + 1, sizeof(unsigned),
                                hipMemcpyDeviceToHost, s));
        LOWD_HIP(hipStreamSynchronize(s));
    });
    if (st == LOWD_OK && unconverged > 0) return LOWD_NOT_CONVERGED;
    return st;
}

lowd_status lowd_batch_solve(int32_t G, const int64_t *node_ptr, const int64_t *edge_ptr,
                             const int32_t *src, const int32_t *dst, int32_t state,
                             int32_t star_max, double tol, int32_t max_sweeps,
                             int32_t check_every, uint8_t *in_set, int64_t *num, int64_t *den,
                             double *D, int32_t *sweeps_used, int32_t *set_sweeps,
                             void *stream) {
    lowd_batch *b = nullptr;
    lowd_status st = lowd_batch_prepare(G, node_ptr, edge_ptr, src, dst, state, star_max, 0, &b,
                                        stream);
    if (st != LOWD_OK) return st;
    std::unique_ptr<lowd_batch, void (*)(lowd_batch *)> guard(b, lowd_batch_free);
    return lowd_batch_solve_prepared(b, tol, max_sweeps, check_every, in_set, num, den, D,
                                     sweeps_used, set_sweeps, stream);
}

}  // extern "C"
