// api.hip -- the C interface (include/lowd.h): argument checks, the solver
// object, device memory, the HIP graph of one sweep, and error reporting.
#include <stdlib.h>
#include <string.h>

#include <exception>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "../../include/lowd.h"
#include "extract.h"
#include "lowd_internal.h"
#include "prune.h"
#include "sweep_state.h"

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
static void validate_graph(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                           const float *w, hipStream_t s) {
    DBuf<int64_t> bad(1);
    launch_validate(n, m, src, dst, w, bad.p, s);
    int64_t b = -1;
    LOWD_HIP(hipMemcpy(&b, bad.p, sizeof(b), hipMemcpyDeviceToHost));
    std::string what = "invalid edge";
    if ((uint64_t)b == ~0ull) {
        b = find_duplicate_pair(n, m, src, dst, s);
        what = "repeated pair";
    }
    if (b >= 0 && (uint64_t)b != ~0ull) {
        int32_t a = 0, c = 0;
        float x = 1.0f;
        LOWD_HIP(hipMemcpy(&a, src + b, 4, hipMemcpyDeviceToHost));
        LOWD_HIP(hipMemcpy(&c, dst + b, 4, hipMemcpyDeviceToHost));
        if (w) LOWD_HIP(hipMemcpy(&x, w + b, 4, hipMemcpyDeviceToHost));
        fail(LOWD_E_GRAPH, what + " at index " + std::to_string(b) + ": (" + std::to_string(a) +
                               ", " + std::to_string(c) + ") weight " + std::to_string(x) +
                               " (n = " + std::to_string(n) + ")");
    }
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
    Csr csr;
    // schedule layout
    DBuf<int32_t> tile_center, tail_nodes;
    DBuf<PhaseDesc> tail_desc;
    DBuf<int64_t> slot_edge, edge_slot;
    DBuf<uint32_t> slot_leaf;
    // state
    DBuf<char> slot_x, L;
    DBuf<float> slot_w;
    DBuf<double> L64, stats_partial, stats_out;
    ExtractScratch ex;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    int32_t ntail = 0;
    ~lowd_solver() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
    }
};

static void reset_state(lowd_solver *sv, hipStream_t s) {
    const int64_t nslots = (int64_t)sv->sch.slot_leaf.size();
    if (nslots > 0)
        sv->fn.init_slots(nslots, sv->slot_edge.p, sv->weighted ? sv->e_w.p : nullptr,
                          sv->slot_x.p, sv->weighted ? sv->slot_w.p : nullptr, s);
    sv->fn.init_loads(sv->n, sv->csr.row_ptr.p, sv->csr.inc.p, sv->weighted ? sv->e_w.p : nullptr,
                      sv->L.p, s);
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
        if (n < 1) fail(LOWD_E_ARG, "n must be >= 1");
        if (m < 0 || m >= ((int64_t)1 << 31)) fail(LOWD_E_ARG, "m must be in [0, 2^31)");
        if (m > 0 && (!src || !dst)) fail(LOWD_E_ARG, "src/dst is NULL");
        if (state != LOWD_STATE_F64 && state != LOWD_STATE_F32K) fail(LOWD_E_ARG, "bad state");
        if (star_max < 1 || star_max > kMaxStar) fail(LOWD_E_ARG, "star_max must be in [1, 16]");
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
        const int64_t lds = (int64_t)lds_capacity_bytes();
        int64_t force = -1;
        if (const char *e = getenv("LOWD_TAIL_SPLIT")) force = atoll(e);
        build_schedule(n, m, hs.data(), hd.data(), star_max, lds, (int64_t)sv->fn.l_bytes, force,
                       sv->sch);
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
        }
        build_incidence(n, m, sv->e_src.p, sv->e_dst.p, sv->csr, s);

        // schedule layout
        upload(sv->tile_center, sc.tile_center, s);
        upload(sv->slot_leaf, sc.slot_leaf, s);
        upload(sv->slot_edge, sc.slot_edge, s);
        upload(sv->edge_slot, sc.edge_slot, s);
        std::vector<PhaseDesc> tdesc(sc.desc.begin() + sc.P0, sc.desc.end());
        upload(sv->tail_desc, tdesc, s);
        upload(sv->tail_nodes, sc.tail_nodes, s);
        sv->ntail = (int32_t)sc.tail_nodes.size();

        // state
        const int64_t nslots = (int64_t)sc.slot_leaf.size();
        sv->slot_x.alloc((size_t)nslots * sv->fn.x_bytes);
        if (sv->weighted) sv->slot_w.alloc((size_t)nslots);
        sv->L.alloc(((size_t)n + 1) * sv->fn.l_bytes);   // [n] = dummy center of empty lanes
        sv->L64.alloc((size_t)n);
        sv->stats_partial.alloc(3 * 1024);
        sv->stats_out.alloc(3);
        reset_state(sv, s);

        // one sweep as a HIP graph: a kernel per whole-GPU phase, then the
        // LDS-resident workgroup for the last phases
        if (sc.P > 0) {
            size_t tail_lds =
                tail_desc_bytes(sc.P - sc.P0) + ((size_t)sv->ntail + 1) * sv->fn.l_bytes;
            if (sc.P0 < sc.P) sv->fn.set_tail_lds(tail_lds);
            hipStream_t cs;
            LOWD_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
            hipError_t err = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
            if (err == hipSuccess) {
                for (int32_t p = 0; p < sc.P0; ++p)
                    sv->fn.phase(sc.desc[(size_t)p], sv->tile_center.p, sv->slot_leaf.p,
                                 sv->slot_x.p, sv->weighted ? sv->slot_w.p : nullptr, sv->L.p,
                                 cs);
                if (sc.P0 < sc.P)
                    sv->fn.tail(sc.P - sc.P0, sv->tail_desc.p, sv->tile_center.p,
                                sv->slot_leaf.p, sv->slot_x.p,
                                sv->weighted ? sv->slot_w.p : nullptr, sv->tail_nodes.p,
                                sv->ntail, sv->L.p, cs);
                err = hipStreamEndCapture(cs, &sv->graph);
            }
            (void)hipStreamDestroy(cs);
            LOWD_HIP(err);
            LOWD_HIP(hipGraphInstantiate(&sv->exec, sv->graph, nullptr, nullptr, 0));
        }
        LOWD_HIP(hipStreamSynchronize(s));
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

static void loads_f64(lowd_solver *sv, hipStream_t s) {
    sv->fn.loads_f64(sv->n, sv->csr.row_ptr.p, sv->csr.inc.p, sv->edge_slot.p, sv->slot_x.p,
                     sv->weighted ? sv->e_w.p : nullptr, sv->L.p, sv->L64.p, s);
}

static void stats(lowd_solver *sv, double out[3], hipStream_t s) {
    int32_t nb = (int32_t)grid_for(sv->n, 256, 1024);
    launch_stats(sv->n, sv->L64.p, sv->stats_partial.p, nb, sv->stats_out.p, s);
    LOWD_HIP(hipGetLastError());
    LOWD_HIP(hipMemcpyAsync(out, sv->stats_out.p, 3 * sizeof(double), hipMemcpyDeviceToHost, s));
    LOWD_HIP(hipStreamSynchronize(s));
}

lowd_status lowd_check(lowd_solver *sv, double *D, double *sum_loads, double *sum_sq_loads,
                       void *stream) {
    return guarded([&] {
        if (!sv) fail(LOWD_E_ARG, "solver is NULL");
        hipStream_t s = (hipStream_t)stream;
        loads_f64(sv, s);
        double o[3];
        stats(sv, o, s);
        if (D) *D = o[0];
        if (sum_loads) *sum_loads = o[1];
        if (sum_sq_loads) *sum_sq_loads = o[2];
    });
}

lowd_status lowd_extract_densest(lowd_solver *sv, uint8_t *in_set, int64_t *num_unit,
                                 double *num_w, int64_t *den, double *D, double *gap,
                                 void *stream) {
    return guarded([&] {
        if (!sv) fail(LOWD_E_ARG, "solver is NULL");
        if (!in_set) fail(LOWD_E_ARG, "in_set is NULL");
        hipStream_t s = (hipStream_t)stream;
        loads_f64(sv, s);
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
        a.in_set = in_set;
        launch_extract(a, sv->ex, s);
        int64_t best[2];
        LOWD_HIP(hipMemcpyAsync(best, sv->ex.best.p, sizeof(best), hipMemcpyDeviceToHost, s));
        double o[3];
        stats(sv, o, s);   // synchronises
        int64_t dn = (int64_t)sv->n - best[0];
        double wnum;
        if (sv->weighted) memcpy(&wnum, &best[1], sizeof(double));
        else wnum = (double)best[1];
        if (num_unit) *num_unit = sv->weighted ? 0 : best[1];
        if (num_w) *num_w = wnum;
        if (den) *den = dn;
        if (D) *D = o[0];
        double rho = wnum / (double)dn;
        if (gap) *gap = rho > 0.0 ? (o[0] - rho) / rho : (o[0] > 0.0 ? 1.0e300 : 0.0);
    });
}

lowd_status lowd_read_state(const lowd_solver *sv, double *x, double *load, void *stream) {
    return guarded([&] {
        if (!sv) fail(LOWD_E_ARG, "solver is NULL");
        hipStream_t s = (hipStream_t)stream;
        if (x && sv->m > 0) sv->fn.read_x(sv->m, sv->edge_slot.p, sv->slot_x.p, x, s);
        if (load) sv->fn.read_loads(sv->n, sv->L.p, load, s);
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
        build_schedule(n, m, src, dst, star_max, 0, 0, -2, sc);
        if (phase && m > 0) memcpy(phase, sc.phase.data(), (size_t)m * 4);
        if (center && m > 0) memcpy(center, sc.center.data(), (size_t)m * 4);
        if (nphases) *nphases = sc.P;
    });
}

lowd_status lowd_solver_info(const lowd_solver *sv, int64_t *info) {
    return guarded([&] {
        if (!sv || !info) fail(LOWD_E_ARG, "NULL argument");
        info[0] = sv->n;
        info[1] = sv->m;
        info[2] = sv->sch.P;
        info[3] = sv->sch.P0;
        info[4] = sv->sch.P - sv->sch.P0;
        info[5] = sv->ntail;
        info[6] = sv->sch.tail_edges;
        info[7] = sv->state;
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
        validate_graph(n, m, src, dst, nullptr, s);
        PruneResult r = run_prune(n, m, src, dst, node_keep, relabel, h_src, h_dst, edge_map, s);
        if (rounds) *rounds = r.rounds;
        if (n_h) *n_h = r.n_h;
        if (m_h) *m_h = r.m_h;
    });
}

lowd_status lowd_batch_solve(int32_t G, const int64_t *node_ptr, const int64_t *edge_ptr,
                             const int32_t *src, const int32_t *dst, int32_t state,
                             int32_t star_max, int32_t sweeps, uint8_t *in_set, int64_t *num,
                             int64_t *den, double *load, void *stream) {
    (void)G; (void)node_ptr; (void)edge_ptr; (void)src; (void)dst; (void)state; (void)star_max;
    (void)sweeps; (void)in_set; (void)num; (void)den; (void)load; (void)stream;
    g_last_error = "lowd_batch_solve is not built yet";
    return LOWD_E_UNSUPPORTED;
}

}  // extern "C"
