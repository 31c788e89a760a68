// schedule.cpp -- the edge schedule of the sweep, computed once on the host.
//
// Algorithm 1 visits the edges in an order it does not fix.  The sweep here
// uses a phase schedule: every phase is a set of vertex-disjoint stars (a
// star = one center node and up to smax leaves, one edge per leaf), so all
// stars of a phase can run at the same time, each as one sequential chain on
// one lane, and the result is exactly that of visiting the phase's edges one
// after another.  A proper edge colouring is the special case smax = 1.
//
// Definition (first fit):
//   center of edge e = its endpoint of larger degree (ties: smaller id);
//   edges are visited in a fixed pseudo-random order: ascending key(e), the
//   e-th output of SplitMix64 seeded with 0, ties by ascending index; e goes
//   to the first phase in which its center is not a leaf and has fewer than
//   smax leaves, and its leaf does not appear at all.
// Sequential order: ascending (phase, edge index).
// The visiting order decides both the phase count (the sweep's cost) and the
// order Algorithm 1 sees the edges in (its convergence per sweep).  On
// power-law graphs a scrambled order reaches the fewest phases found (as
// many as visiting the most constrained leaves first) while converging in
// fewer sweeps than any structured order tried: on a 1M-node, 10M-edge
// Chung-Lu graph 22 sweeps to a 1e-6 gap against 26 in index order and 38
// with the most constrained leaves first.
//
// Device layout: within a phase the stars are sorted by size (descending,
// then center id) and dealt to tiles of 64, one star per lane; row k of the
// phase holds the k-th leaf of every tile deeper than k (see PhaseDesc), so
// a row is one coalesced 64-wide access and every address follows from the
// phase descriptor.
//
// The last phases of a power-law graph are small and touch few nodes (the
// dense core); the schedule picks a split phase P0 such that the nodes of
// phases [P0, P) fit in one workgroup's LDS, and those phases run inside a
// single workgroup separated by LDS barriers instead of kernel boundaries.
#include <stdint.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <exception>
#include <memory>
#include <numeric>
#include <thread>
#include <utility>
#include <vector>

#include "lowd_internal.h"

namespace lowd {

namespace {

struct Bits {
    std::vector<uint64_t> w;
    inline uint64_t word(size_t i) const { return i < w.size() ? w[i] : 0ull; }
    inline void set(int32_t p) {
        size_t i = (size_t)p >> 6;
        if (i >= w.size()) w.resize(i + 1 + (i >> 1), 0ull);
        w[i] |= 1ull << (p & 63);
    }
};

// An array of trivially constructible elements left uninitialised: every
// use below writes each element before reading it, so large temporaries are
// not first cleared on one thread.
template <class T>
struct Raw {
    std::unique_ptr<T[]> p;
    size_t n = 0;
    Raw() = default;
    explicit Raw(size_t k) : p(new T[k > 0 ? k : 1]), n(k) {}
    T &operator[](size_t i) { return p[i]; }
    const T &operator[](size_t i) const { return p[i]; }
    T *data() { return p.get(); }
    size_t size() const { return n; }
    void swap(Raw &o) {
        std::swap(p, o.p);
        std::swap(n, o.n);
    }
    void reset() {
        p.reset();
        n = 0;
    }
};

// The e-th output (e = 0, 1, ...) of SplitMix64 (Steele, Lea and Flood,
// "Fast splittable pseudorandom number generators", OOPSLA 2014) seeded
// with 0: the state after e + 1 steps of adding the golden-ratio increment,
// through the generator's output mix.
inline uint64_t visit_key(int64_t e) {
    uint64_t z = (uint64_t)(e + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Host threads for the schedule (LOWD_HOST_THREADS overrides; at most 16).
// Every parallel step below writes disjoint entries or reduces in a fixed
// order, so the schedule is the same for any thread count.
int host_threads() {
    static const int t = [] {
        int k = (int)std::thread::hardware_concurrency();
        if (const char *e = getenv("LOWD_HOST_THREADS")) k = atoi(e);
        return std::max(1, std::min(k, 16));
    }();
    return t;
}

// f(t) on T threads; an exception in any of them is rethrown here
template <class F>
void run_threads(int T, F &&f) {
    if (T <= 1) {
        f(0);
        return;
    }
    std::vector<std::thread> th;
    std::vector<std::exception_ptr> err((size_t)T);
    for (int t = 0; t < T; ++t)
        th.emplace_back([&, t] {
            try {
                f(t);
            } catch (...) {
                err[(size_t)t] = std::current_exception();
            }
        });
    for (auto &x : th) x.join();
    for (auto &e : err)
        if (e) std::rethrow_exception(e);
}

// threads for a step over `work` items: one per 64K items, at most
// host_threads() (small graphs, such as a batch's, stay on the caller's
// thread)
int threads_for(int64_t work) {
    return (int)std::max<int64_t>(1, std::min<int64_t>(host_threads(), work / 65536));
}

// f(t, lo, hi) over T contiguous chunks of [0, n)
template <class F>
void parallel_chunks(int64_t n, F &&f) {
    const int T = threads_for(n);
    run_threads(T, [&](int t) { f(t, n * t / T, n * (t + 1) / T); });
}

// f(i) for i in [0, n), items taken one at a time from a shared counter
// (items of very uneven cost); parallel only when `work` is large
template <class F>
void parallel_items(int64_t n, int64_t work, F &&f) {
    const int T = (int)std::max<int64_t>(1, std::min<int64_t>(threads_for(work), n));
    std::atomic<int64_t> next(0);
    run_threads(T, [&](int) {
        for (int64_t i = next++; i < n; i = next++) f(i);
    });
}

// f(lo, hi) over the nodes [0, n) in blocks of 1024 (per-node work of very
// uneven cost: a node's work follows its degree)
template <class F>
void parallel_nodes(int32_t n, int64_t work, F &&f) {
    constexpr int64_t kBlock = 1024;
    parallel_items(((int64_t)n + kBlock - 1) / kBlock, work, [&](int64_t b) {
        f((int32_t)(b * kBlock), (int32_t)std::min<int64_t>((b + 1) * kBlock, n));
    });
}

// Edge indices 0..m-1 in ascending visit_key order.  The keys are distinct
// (SplitMix64's output is a bijection of its state, and the states of
// distinct e differ), so the order is total.  Parallel: the edges are dealt
// to 4096 buckets by their top 12 key bits (per-thread counts, one scan,
// per-thread scatter), then every bucket is sorted on its own.
Raw<int64_t> sort_by_visit_key(int64_t m) {
    constexpr int kTop = 12;
    constexpr size_t kB = (size_t)1 << kTop;
    struct KV {
        uint64_t k;
        int64_t e;
    };
    Raw<KV> kv((size_t)m);
    const int T = threads_for(m);
    std::vector<int64_t> cnt((size_t)T * kB, 0);
    run_threads(T, [&](int t) {
        int64_t *c = cnt.data() + (size_t)t * kB;
        for (int64_t e = m * t / T; e < m * (t + 1) / T; ++e) ++c[visit_key(e) >> (64 - kTop)];
    });
    std::vector<int64_t> bstart(kB + 1, 0);
    {
        int64_t run = 0;
        for (size_t b = 0; b < kB; ++b) {
            bstart[b] = run;
            for (int t = 0; t < T; ++t) {
                const int64_t c = cnt[(size_t)t * kB + b];
                cnt[(size_t)t * kB + b] = run;
                run += c;
            }
        }
        bstart[kB] = run;
    }
    run_threads(T, [&](int t) {
        int64_t *c = cnt.data() + (size_t)t * kB;
        for (int64_t e = m * t / T; e < m * (t + 1) / T; ++e) {
            const uint64_t k = visit_key(e);
            kv[(size_t)c[k >> (64 - kTop)]++] = KV{k, e};
        }
    });
    parallel_items((int64_t)kB, m, [&](int64_t b) {
        std::sort(kv.data() + bstart[(size_t)b], kv.data() + bstart[(size_t)b + 1],
                  [](const KV &x, const KV &y) { return x.k < y.k; });
    });
    Raw<int64_t> idx((size_t)m);
    parallel_chunks(m, [&](int, int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) idx[(size_t)i] = kv[(size_t)i].e;
    });
    return idx;
}

// bits needed to hold 0 .. k-1
int bits_for(int64_t k) {
    int b = 0;
    while (b < 63 && ((int64_t)1 << b) < k) ++b;
    return b;
}

// Stable LSD radix sort of the pairs (key[i], val[i]) by key bits [0, bits),
// 8 bits a pass: per-thread digit counts over contiguous ranges, one scan in
// (digit, thread) order, per-thread scatter.  A pass whose digit is the same
// for every key is skipped.
void radix_sort_kv(Raw<uint64_t> &key, Raw<uint32_t> &val, int bits) {
    constexpr int kD = 8;
    constexpr size_t kB = (size_t)1 << kD;
    const int64_t n = (int64_t)key.size();
    const int T = threads_for(n);
    std::vector<int64_t> cnt((size_t)T * kB);
    Raw<uint64_t> k2;
    Raw<uint32_t> v2;
    for (int shift = 0; shift < bits; shift += kD) {
        std::fill(cnt.begin(), cnt.end(), 0);
        run_threads(T, [&](int t) {
            int64_t *c = cnt.data() + (size_t)t * kB;
            for (int64_t i = n * t / T; i < n * (t + 1) / T; ++i) ++c[(key[(size_t)i] >> shift) & (kB - 1)];
        });
        int64_t run = 0;
        bool one_digit = false;
        for (size_t d = 0; d < kB; ++d) {
            int64_t total = 0;
            for (int t = 0; t < T; ++t) {
                const int64_t c = cnt[(size_t)t * kB + d];
                cnt[(size_t)t * kB + d] = run;
                run += c;
                total += c;
            }
            if (total == n) one_digit = true;
        }
        if (one_digit) continue;
        if (k2.size() == 0) {
            Raw<uint64_t>((size_t)n).swap(k2);
            Raw<uint32_t>((size_t)n).swap(v2);
        }
        run_threads(T, [&](int t) {
            int64_t *c = cnt.data() + (size_t)t * kB;
            for (int64_t i = n * t / T; i < n * (t + 1) / T; ++i) {
                const size_t to = (size_t)c[(key[(size_t)i] >> shift) & (kB - 1)]++;
                k2[to] = key[(size_t)i];
                v2[to] = val[(size_t)i];
            }
        });
        key.swap(k2);
        val.swap(v2);
    }
}

// Per-phase cost model (microseconds) used to place the split P0.  A phase
// run by a whole-GPU launch costs one kernel boundary inside a HIP graph plus
// its streamed bytes; a phase inside the LDS-resident workgroup costs a
// barrier plus its longest star chain plus one CU's streaming time.
struct CostModel {
    double grid_fixed_us = 3.9;                  // launch, one round trip, chain, stores
    double grid_us_per_edge = 48.0 / 4.0e6;      // ~48 B per edge at ~4 TB/s
    double mid_fixed_us = 3.8;                   // barrier + gathers through one CU
    double mid_us_per_round = 1.2;               // each further tile per wave (no prefetch)
    double mid_us_per_edge = 0.0018;             // ~4 random cache lines per edge, one CU
    double tail_fixed_us = 1.0;                  // barrier + LDS gathers
    double us_per_depth = 0.06;                  // one dependent step of a star chain
    double serial_us_per_edge = 24.0 / 1.0e5;    // ~24 B per edge at ~100 GB/s (one CU)
};

}  // namespace

void build_schedule(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, int32_t smax,
                    int64_t lds_bytes, int64_t l_bytes, int64_t force_p0, int64_t force_p1,
                    Schedule &out, bool whole_in_lds, int64_t pull_min_edges) {
    out = Schedule();
    if (smax > kMaxStar && force_p0 != -2) {
        // the device layout holds stars of up to kMaxStar leaves; callers that
        // only want the phase assignment pass force_p0 = -2
        fail(LOWD_E_ARG, "star_max must be at most 32 for the sweep kernels");
    }
    if (m >= (int64_t)kNoStation)
        fail(LOWD_E_UNSUPPORTED, "graph too large for 31-bit station indices");
    out.n = n;
    out.m = m;
    out.smax = smax;

    // ---- orientation and visiting order ------------------------------------
    std::vector<int32_t> deg((size_t)n, 0);
    parallel_chunks(m, [&](int, int64_t lo, int64_t hi) {
        for (int64_t e = lo; e < hi; ++e) {
            __atomic_fetch_add(&deg[(size_t)src[e]], 1, __ATOMIC_RELAXED);
            __atomic_fetch_add(&deg[(size_t)dst[e]], 1, __ATOMIC_RELAXED);
        }
    });
    std::vector<int32_t> ctr((size_t)m);
    parallel_chunks(m, [&](int, int64_t lo, int64_t hi) {
        for (int64_t e = lo; e < hi; ++e) {
            const int32_t a = src[e], b = dst[e];
            const bool a_center = deg[(size_t)a] > deg[(size_t)b] ||
                                  (deg[(size_t)a] == deg[(size_t)b] && a < b);
            ctr[(size_t)e] = a_center ? a : b;
        }
    });
    const Raw<int64_t> visit = sort_by_visit_key(m);
    // the edges' centers and leaves in visiting order
    Raw<int32_t> cv((size_t)m), lv((size_t)m);
    parallel_chunks(m, [&](int, int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) {
            const int64_t e = visit[(size_t)i];
            cv[(size_t)i] = ctr[(size_t)e];
            lv[(size_t)i] = src[e] == ctr[(size_t)e] ? dst[e] : src[e];
        }
    });

    // ---- per-node incidence lists ------------------------------------------
    // Every visiting position i is on two nodes: entry 2 i is its center,
    // 2 i + 1 its leaf.  Sorted stably by node, a node's entries come in
    // ascending position, at [off[v], off[v+1]).  The phase of position i
    // depends only on the roles its nodes took at earlier positions: rc[i] /
    // rl[i] = how many earlier positions its center / its leaf is on.
    std::vector<int64_t> off((size_t)n + 1, 0);
    for (int32_t v = 0; v < n; ++v) off[(size_t)v + 1] = off[(size_t)v] + deg[(size_t)v];
    std::vector<int32_t>().swap(deg);
    Raw<uint32_t> rc((size_t)m), rl((size_t)m);
    {
        Raw<uint64_t> key((size_t)(2 * m));
        Raw<uint32_t> val((size_t)(2 * m));
        parallel_chunks(m, [&](int, int64_t lo, int64_t hi) {
            for (int64_t i = lo; i < hi; ++i) {
                key[(size_t)(2 * i)] = (uint64_t)cv[(size_t)i];
                key[(size_t)(2 * i + 1)] = (uint64_t)lv[(size_t)i];
                val[(size_t)(2 * i)] = (uint32_t)(2 * i);
                val[(size_t)(2 * i + 1)] = (uint32_t)(2 * i + 1);
            }
        });
        radix_sort_kv(key, val, bits_for(n));
        parallel_chunks(2 * m, [&](int, int64_t lo, int64_t hi) {
            for (int64_t j = lo; j < hi; ++j) {
                const uint32_t x = val[(size_t)j];
                (x & 1u ? rl : rc)[(size_t)(x >> 1)] = (uint32_t)(j - off[(size_t)key[(size_t)j]]);
            }
        });
    }

    // ---- first fit ----------------------------------------------------------
    // One cache line per node: used = phases 0..63 where the node has any
    // role, noc = phases 0..63 where it cannot be a center (it is a leaf
    // there, or its star is full), done = how many of its positions are
    // placed, cnt = its star sizes in phases 0..kCntInline-1.  Later phases,
    // which only high-degree nodes reach, live in per-node overflow storage.
    constexpr int kCntInline = 44;
    struct alignas(64) NodeState {
        uint64_t used, noc;
        uint32_t done;
        uint8_t cnt[kCntInline];
    };
    static_assert(sizeof(NodeState) == 64, "one cache line per node");
    struct Overflow {
        Bits used, noc;             // phases 64, 65, ...
        std::vector<uint8_t> cnt;   // star sizes of phases kCntInline, kCntInline + 1, ...
    };
    std::unique_ptr<NodeState[]> ns(new NodeState[(size_t)n + 1]);
    parallel_chunks(n, [&](int, int64_t lo, int64_t hi) {
        memset((void *)(ns.get() + lo), 0, (size_t)(hi - lo) * sizeof(NodeState));
    });
    std::vector<std::unique_ptr<Overflow>> ov((size_t)n);
    auto over = [&](int32_t u) -> Overflow & {
        if (!ov[(size_t)u]) ov[(size_t)u].reset(new Overflow());
        return *ov[(size_t)u];
    };
    auto busy_word = [&](int32_t c, int32_t l, size_t wi) -> uint64_t {
        if (wi == 0) return ns[(size_t)c].noc | ns[(size_t)l].used;
        const Overflow *oc = ov[(size_t)c].get(), *ol = ov[(size_t)l].get();
        return (oc ? oc->noc.word(wi - 1) : 0ull) | (ol ? ol->used.word(wi - 1) : 0ull);
    };
    Raw<int32_t> pv((size_t)m);
    // is position i next in line at both of its nodes?
    auto ready = [&](int64_t i) {
        return __atomic_load_n(&ns[(size_t)cv[(size_t)i]].done, __ATOMIC_ACQUIRE) == rc[(size_t)i] &&
               __atomic_load_n(&ns[(size_t)lv[(size_t)i]].done, __ATOMIC_ACQUIRE) == rl[(size_t)i];
    };
    // place position i: its phase from the state of its two nodes, which then
    // take their roles in it
    auto place = [&](int64_t i) -> int32_t {
        const int32_t c = cv[(size_t)i], l = lv[(size_t)i];
        NodeState &sc = ns[(size_t)c], &sl = ns[(size_t)l];
        int32_t p = 0;
        for (size_t wi = 0;; ++wi) {
            const uint64_t busy = busy_word(c, l, wi);
            if (~busy) {
                p = (int32_t)(wi * 64 + (size_t)__builtin_ctzll(~busy));
                break;
            }
        }
        uint8_t *cc;
        if (p < kCntInline) {
            cc = &sc.cnt[p];
        } else {
            std::vector<uint8_t> &oc = over(c).cnt;
            const size_t q = (size_t)(p - kCntInline);
            if (q >= oc.size()) oc.resize(q + 1 + (q >> 1), 0);
            cc = &oc[q];
        }
        const bool full = ++*cc >= smax;
        if (p < 64) {
            const uint64_t bit = 1ull << p;
            sc.used |= bit;
            sl.used |= bit;
            sl.noc |= bit;
            if (full) sc.noc |= bit;
        } else {
            const int32_t q = p - 64;
            Overflow &oc = over(c);
            oc.used.set(q);
            if (full) oc.noc.set(q);
            Overflow &ol = over(l);
            ol.used.set(q);
            ol.noc.set(q);
        }
        pv[(size_t)i] = p;
        __atomic_store_n(&sc.done, sc.done + 1, __ATOMIC_RELEASE);
        __atomic_store_n(&sl.done, sl.done + 1, __ATOMIC_RELEASE);
        return p;
    };
    // Threads claim positions in ascending chunks of 64 and place a position
    // once every earlier position at both of its nodes is placed; a position
    // that is not ready waits in a short per-thread list, retried before each
    // new position, while the thread goes on.  Every node's state thus
    // changes in visiting order and each position sees exactly the state the
    // sequential loop would give it (the acquire / release pairs on `done`
    // order the state between threads).  The lowest unplaced position is
    // always ready, so the placement always progresses.
    const int T_ff = threads_for(m);
    std::vector<int32_t> p_of_thread((size_t)T_ff, 0);
    std::atomic<int64_t> next_chunk(0);
    run_threads(T_ff, [&](int t) {
        constexpr int64_t kChunk = 64, kAhead = 8;
        constexpr size_t kMaxPending = 32;
        int32_t pend[kMaxPending];
        size_t np = 0;
        int32_t pmax = 0;
        auto retry = [&] {
            size_t w = 0;
            for (size_t k = 0; k < np; ++k) {
                if (ready(pend[k])) pmax = std::max(pmax, place(pend[k]) + 1);
                else pend[w++] = pend[k];
            }
            np = w;
        };
        for (int64_t c0 = next_chunk.fetch_add(kChunk); c0 < m; c0 = next_chunk.fetch_add(kChunk)) {
            const int64_t c1 = std::min(c0 + kChunk, m);
            for (int64_t i = c0; i < c1; ++i) {
                if (i + kAhead < c1) {
                    __builtin_prefetch(&ns[(size_t)cv[(size_t)(i + kAhead)]]);
                    __builtin_prefetch(&ns[(size_t)lv[(size_t)(i + kAhead)]]);
                }
                retry();
                while (np == kMaxPending) {
                    __builtin_ia32_pause();
                    retry();
                }
                if (ready(i)) pmax = std::max(pmax, place(i) + 1);
                else pend[np++] = (int32_t)i;
            }
        }
        retry();
        while (np > 0) {
            __builtin_ia32_pause();
            retry();
        }
        p_of_thread[(size_t)t] = pmax;
    });
    int32_t P = 0;
    for (const int32_t x : p_of_thread) P = std::max(P, x);
    out.P = P;
    out.phase.resize((size_t)m);
    parallel_chunks(m, [&](int, int64_t lo, int64_t hi) {
        for (int64_t i = lo; i < hi; ++i) out.phase[(size_t)visit[(size_t)i]] = pv[(size_t)i];
    });
    out.center = std::move(ctr);
    ns.reset();
    rc.reset();
    rl.reset();
    lv.reset();
    std::vector<std::unique_ptr<Overflow>>().swap(ov);

    if (force_p0 == -2) return;   // phase assignment only

    // ---- stars --------------------------------------------------------------
    // Every edge is on two nodes; its entries (node, phase) sorted stably
    // from edge order put each node's edges in ascending (phase, edge index)
    // at [off[v], off[v+1]): at[j] = the edge, ph[j] = its phase, cen[j] =
    // whether the node is its center.  A node has one role per phase, so a
    // run of equal phases is either one edge the node is the leaf of or the
    // star it is the center of (its edges in ascending index).  last[v] = v's
    // last phase.
    const int pbits = bits_for(P);
    Raw<uint32_t> at((size_t)(2 * m));
    Raw<int32_t> ph((size_t)(2 * m));
    Raw<uint8_t> cen((size_t)(2 * m));
    {
        Raw<uint64_t> key((size_t)(2 * m));
        parallel_chunks(m, [&](int, int64_t lo, int64_t hi) {
            for (int64_t e = lo; e < hi; ++e) {
                const uint64_t p = (uint64_t)out.phase[(size_t)e];
                const bool src_center = out.center[(size_t)e] == src[e];
                key[(size_t)(2 * e)] = ((uint64_t)src[e] << pbits) | p;
                key[(size_t)(2 * e + 1)] = ((uint64_t)dst[e] << pbits) | p;
                at[(size_t)(2 * e)] = (uint32_t)e | (src_center ? 0x80000000u : 0u);
                at[(size_t)(2 * e + 1)] = (uint32_t)e | (src_center ? 0u : 0x80000000u);
            }
        });
        radix_sort_kv(key, at, bits_for(n) + pbits);
        parallel_chunks(2 * m, [&](int, int64_t lo, int64_t hi) {
            for (int64_t j = lo; j < hi; ++j) {
                ph[(size_t)j] = (int32_t)(key[(size_t)j] & (((uint64_t)1 << pbits) - 1));
                cen[(size_t)j] = (uint8_t)(at[(size_t)j] >> 31);
                at[(size_t)j] &= 0x7FFFFFFFu;
            }
        });
    }
    std::vector<int32_t> last((size_t)n, -1);
    parallel_chunks(n, [&](int, int64_t lo, int64_t hi) {
        for (int64_t v = lo; v < hi; ++v)
            if (off[(size_t)v + 1] > off[(size_t)v]) last[(size_t)v] = ph[(size_t)off[(size_t)v + 1] - 1];
    });
    // Stars of phase p, sorted by size (descending) then center, at
    // star[pstar[p] .. pstar[p+1]).  Threads own contiguous node ranges of
    // about equal incidence; each counts its stars per (phase, size), one
    // scan in (phase, size descending, thread) order gives every thread its
    // write offsets, and each writes its stars in ascending center order.
    struct Star { int64_t begin; int32_t len; int32_t center; };   // begin: into at[]
    const int64_t bins = (int64_t)P * smax;
    const int T_st = (int)std::max<int64_t>(
        1, std::min<int64_t>(threads_for(2 * m), (int64_t)(64 << 20) / std::max<int64_t>(bins, 1)));
    std::vector<int32_t> vfrom((size_t)T_st + 1, n);
    for (int t = 0; t < T_st; ++t)
        vfrom[(size_t)t] = (int32_t)(std::lower_bound(off.begin(), off.end() - 1, 2 * m * t / T_st) -
                                     off.begin());
    auto for_stars = [&](int t, auto &&g) {   // g(v, begin, len, phase) over thread t's stars
        for (int32_t v = vfrom[(size_t)t]; v < vfrom[(size_t)t + 1]; ++v) {
            const int64_t b = off[(size_t)v + 1];
            for (int64_t j = off[(size_t)v]; j < b;) {
                const int32_t p = ph[(size_t)j];
                int64_t k = j + 1;
                while (k < b && ph[(size_t)k] == p) ++k;
                if (cen[(size_t)j]) g(v, j, (int32_t)(k - j), p);
                j = k;
            }
        }
    };
    std::vector<int64_t> scnt((size_t)T_st * (size_t)bins, 0);
    run_threads(T_st, [&](int t) {
        int64_t *c = scnt.data() + (size_t)t * bins;
        for_stars(t, [&](int32_t, int64_t, int32_t len, int32_t p) { ++c[(int64_t)p * smax + len - 1]; });
    });
    std::vector<int64_t> pstar((size_t)P + 1, 0), ecount((size_t)P, 0), maxstar((size_t)P, 0);
    {
        int64_t run = 0;
        for (int32_t p = 0; p < P; ++p) {
            pstar[(size_t)p] = run;
            for (int32_t len = smax; len >= 1; --len)
                for (int t = 0; t < T_st; ++t) {
                    int64_t &c = scnt[(size_t)t * bins + (size_t)p * smax + len - 1];
                    if (c > 0) {
                        ecount[(size_t)p] += c * len;
                        maxstar[(size_t)p] = std::max<int64_t>(maxstar[(size_t)p], len);
                    }
                    const int64_t k = c;
                    c = run;
                    run += k;
                }
        }
        pstar[(size_t)P] = run;
    }
    std::vector<Star> star((size_t)pstar[(size_t)P]);
    run_threads(T_st, [&](int t) {
        int64_t *c = scnt.data() + (size_t)t * bins;
        for_stars(t, [&](int32_t v, int64_t j, int32_t len, int32_t p) {
            star[(size_t)c[(int64_t)p * smax + len - 1]++] = Star{j, len, v};
        });
    });
    std::vector<int64_t>().swap(scnt);
    auto nstars = [&](int32_t p) { return pstar[(size_t)p + 1] - pstar[(size_t)p]; };

    // ---- split P0 -----------------------------------------------------------
    std::vector<int64_t> nodes_from((size_t)P + 2, 0);   // nodes with last >= p
    for (int32_t u = 0; u < n; ++u)
        if (last[(size_t)u] >= 0) ++nodes_from[(size_t)last[(size_t)u]];
    for (int32_t p = P - 1; p >= 0; --p) nodes_from[(size_t)p] += nodes_from[(size_t)p + 1];
    CostModel cm;
    // the tail [p0, P) fits when its descriptors and node loads fit in LDS,
    // and no tail phase is wider than the workgroup
    // and no tail or middle phase has a star deeper than the tiers' tiles
    int32_t min_p0 = 0, min_p1 = 0;
    for (int32_t p = 0; p < P; ++p) {
        if (nstars(p) > (int64_t)kTailWaves * kWave) min_p0 = p + 1;
        if (maxstar[(size_t)p] > kTierStar) {
            min_p0 = std::max(min_p0, p + 1);
            min_p1 = p + 1;
        }
    }
    auto fits = [&](int32_t p0) {
        if (lds_bytes <= 0) return p0 >= P;
        if (p0 < min_p0) return false;
        return (int64_t)tail_desc_bytes(P - p0) + (nodes_from[(size_t)p0] + 2) * l_bytes <= lds_bytes;
    };
    // the middle tier keeps only its descriptors in LDS
    const int64_t max_mid = lds_bytes > 0 ? lds_bytes / (int64_t)sizeof(PhaseDesc) - 1 : 0;
    std::vector<double> gpre((size_t)P + 1, 0.0), mpre((size_t)P + 1, 0.0), tsuf((size_t)P + 1, 0.0);
    for (int32_t p = 0; p < P; ++p) {
        const double tiles = (double)((nstars(p) + kWave - 1) / kWave);
        const double rounds = std::ceil(tiles / kTailWaves);
        gpre[(size_t)p + 1] = gpre[(size_t)p] + cm.grid_fixed_us +
                              cm.grid_us_per_edge * (double)ecount[(size_t)p];
        mpre[(size_t)p + 1] = mpre[(size_t)p] + cm.mid_fixed_us +
                              cm.mid_us_per_round * (rounds > 1 ? rounds - 1 : 0) +
                              cm.us_per_depth * (double)maxstar[(size_t)p] * rounds +
                              cm.mid_us_per_edge * (double)ecount[(size_t)p];
    }
    for (int32_t p = P - 1; p >= 0; --p)
        tsuf[(size_t)p] = tsuf[(size_t)p + 1] + cm.tail_fixed_us +
                          cm.us_per_depth * (double)maxstar[(size_t)p] +
                          cm.serial_us_per_edge * (double)ecount[(size_t)p];
    // best P1 <= p0 for the middle tier: min over p1 of gpre[p1] - mpre[p1]
    auto best_p1 = [&](int32_t p0, double *cost) {
        int32_t b = p0;
        double bc = gpre[(size_t)p0] - mpre[(size_t)p0];
        for (int32_t p1 = p0 - 1; p1 >= min_p1 && p0 - p1 <= max_mid; --p1) {
            const double c = gpre[(size_t)p1] - mpre[(size_t)p1];
            if (c < bc) { bc = c; b = p1; }
        }
        *cost = bc + mpre[(size_t)p0];
        return b;
    };
    int32_t P0 = P, P1 = P;
    if (whole_in_lds) {
        P0 = 0;
        P1 = 0;
    } else if (force_p0 >= 0 || force_p1 >= 0) {
        P0 = (int32_t)std::min<int64_t>(force_p0 >= 0 ? force_p0 : P, P);
        while (P0 < P && !fits(P0)) ++P0;
        P1 = (int32_t)std::min<int64_t>(force_p1 >= 0 ? force_p1 : P0, P0);
        if (lds_bytes <= 0) P1 = P0;
        if (P0 - P1 > max_mid) P1 = (int32_t)(P0 - max_mid);
        if (P1 < min_p1) P1 = std::min(min_p1, P0);
    } else if (lds_bytes > 0 && P > 0) {
        double c0;
        P1 = best_p1(P, &c0);
        double best = c0;
        for (int32_t p0 = P - 1; p0 >= 0; --p0) {
            if (!fits(p0)) break;   // fits(p0) implies fits(p0 + 1)
            double c;
            int32_t p1 = best_p1(p0, &c);
            c += tsuf[(size_t)p0];
            if (c < best) { best = c; P0 = p0; P1 = p1; }
        }
    }
    out.P1 = P1;
    out.P0 = P0;

    // tail node ids (ascending) -> local index
    std::vector<int32_t> local((size_t)n, -1);
    if (whole_in_lds) {
        for (int32_t u = 0; u < n; ++u) {
            local[(size_t)u] = u;
            out.tail_nodes.push_back(u);
        }
    } else if (P0 < P) {
        for (int32_t u = 0; u < n; ++u)
            if (last[(size_t)u] >= P0) {
                local[(size_t)u] = (int32_t)out.tail_nodes.size();
                out.tail_nodes.push_back(u);
            }
    }


    // ---- tiles and slots ----------------------------------------------------
    out.desc.assign((size_t)P, PhaseDescWide{});
    out.phase_edges = ecount;
    out.phase_depth.assign((size_t)P, 0);
    std::vector<int64_t> pslots((size_t)P, 0);
    parallel_items(P, m, [&](int64_t pp) {
        const int32_t p = (int32_t)pp;
        PhaseDescWide &d = out.desc[(size_t)p];
        const int64_t t = (nstars(p) + kWave - 1) / kWave;
        for (int k = 0; k < kMaxStar; ++k) d.T[k] = 0;
        for (int64_t i = 0; i < t; ++i) {
            // tiles whose first (deepest) star is longer than k
            const int32_t len = star[(size_t)(pstar[(size_t)p] + i * kWave)].len;
            for (int k = 0; k < len; ++k) ++d.T[k];
        }
        for (int k = 0; k < kMaxStar; ++k) pslots[(size_t)p] += (int64_t)d.T[k] * kWave;
        out.phase_depth[(size_t)p] = t > 0 ? star[(size_t)pstar[(size_t)p]].len : 0;
    });
    int64_t ntiles = 0, nslots = 0;
    for (int32_t p = 0; p < P; ++p) {
        PhaseDescWide &d = out.desc[(size_t)p];
        d.slot_base = nslots;
        d.tile0 = (int32_t)ntiles;
        d.sink = 0;
        nslots += pslots[(size_t)p];
        ntiles += (nstars(p) + kWave - 1) / kWave;
    }
    // lanes without a star get the dummy node: n (whole-GPU phases) or the
    // tail's LDS entry after its nodes
    out.tile_center.assign((size_t)ntiles * kWave, n);
    out.slot_leaf.assign((size_t)nslots, (uint32_t)n + 1u);   // padding: the infinite dummy
    out.slot_edge.assign((size_t)nslots, -1);
    out.edge_slot.assign((size_t)m, -1);
    const int32_t ntail_nodes = (int32_t)out.tail_nodes.size();
    // stations: slots [0, nslots), lanes after them, then the tail's nodes
    out.center_base = nslots;
    out.tail_base = nslots + ntiles * kWave;
    out.slot_next.assign((size_t)nslots, kNoStation);
    out.center_next.assign((size_t)ntiles * kWave, kNoStation);
    out.tail_next.assign((size_t)ntail_nodes, kNoStation);
    for (int32_t p = P0; p < P; ++p) {
        out.tail_edges += ecount[(size_t)p];
        // tail dummies are the LDS entries after the tail's nodes
        const PhaseDescWide &d = out.desc[(size_t)p];
        const int64_t t = (nstars(p) + kWave - 1) / kWave;
        for (int64_t i = 0; i < t * kWave; ++i)
            out.tile_center[(size_t)(d.tile0 * kWave + i)] = ntail_nodes;
        for (int64_t i = 0; i < pslots[(size_t)p]; ++i)
            out.slot_leaf[(size_t)(d.slot_base + i)] = (uint32_t)ntail_nodes + 1u;
    }
    // the lane station of each whole-GPU star's center, at the star's first
    // entry in its center's list
    Raw<uint32_t> lane_station((size_t)(2 * m));
    // stars in chunks of 16384 (a phase can hold most of the edges)
    constexpr int64_t kStarChunk = 16384;
    std::vector<std::pair<int32_t, int64_t>> chunks;
    for (int32_t p = 0; p < P; ++p)
        for (int64_t i = 0; i < nstars(p); i += kStarChunk) chunks.emplace_back(p, i);
    parallel_items((int64_t)chunks.size(), m, [&](int64_t ci) {
        const int32_t p = chunks[(size_t)ci].first;
        const bool tail = p >= P0;
        const PhaseDescWide &d = out.desc[(size_t)p];
        const int64_t i0 = chunks[(size_t)ci].second, i1 = std::min(i0 + kStarChunk, nstars(p));
        for (int64_t i = i0; i < i1; ++i) {
            const Star &sr = star[(size_t)(pstar[(size_t)p] + i)];
            const int64_t tt = i / kWave;
            const int lane = (int)(i % kWave);
            int64_t rows_before = 0;   // sum_k min(T[k], tt)
            for (int k = 0; k < kMaxStar; ++k) rows_before += std::min<int64_t>(d.T[k], tt);
            const int64_t tile_base = d.slot_base + rows_before * kWave;
            const int64_t lane_at = (d.tile0 + tt) * kWave + lane;
            out.tile_center[(size_t)lane_at] = tail ? local[(size_t)sr.center] : sr.center;
            if (!tail) lane_station[(size_t)sr.begin] = (uint32_t)(out.center_base + lane_at);
            for (int32_t k = 0; k < sr.len; ++k) {
                const int64_t e = at[(size_t)(sr.begin + k)];
                const bool c_is_dst = dst[e] == sr.center;
                const int32_t leaf = c_is_dst ? src[e] : dst[e];
                const int32_t id = tail ? local[(size_t)leaf] : leaf;
                const int64_t sl = tile_base + (int64_t)k * kWave + lane;
                out.slot_leaf[(size_t)sl] = (uint32_t)id | (c_is_dst ? kCenterIsDst : 0u);
                out.slot_edge[(size_t)sl] = e;
                out.edge_slot[(size_t)e] = sl;
            }
        }
    });
    std::vector<Star>().swap(star);

    // ---- stations -----------------------------------------------------------
    // Each node's stations in sweep order: one per whole-GPU phase it takes
    // part in (its lane as a center, its slot as a leaf), then its tail
    // entry; each names where its updated load goes, the last one wrapping
    // to the first.  A station of a pushed phase is where the node's load
    // waits for it: its predecessor writes there.  A station of a pulled
    // phase (a whole-GPU phase of at least pull_min_edges edges) instead
    // reads the load from its predecessor's station, which keeps its own
    // output: coalesced writes and random reads, where pushing scatters the
    // writes.  Nodes on no edge get a home entry of their own, numbered in
    // node order after the tail's entries.
    std::vector<uint8_t> pulled((size_t)P, 0);
    bool any_pull = false;
    if (pull_min_edges >= 0)
        for (int32_t p = 0; p < P1; ++p)
            if (out.phase_edges[(size_t)p] >= pull_min_edges) pulled[(size_t)p] = 1, any_pull = true;
    if (any_pull) {
        out.pull.assign(pulled.begin(), pulled.end());
        // rows and lanes of a pulled phase read their own entries unless a
        // node's predecessor is named below (padding rows keep +inf there,
        // empty lanes 0)
        out.slot_src.resize((size_t)nslots);
        out.center_src.resize(out.center_next.size());
        for (int32_t p = 0; p < P1; ++p) {
            if (!pulled[(size_t)p]) continue;
            const PhaseDescWide &d = out.desc[(size_t)p];
            int64_t rows = 0;
            for (int k = 0; k < kMaxStar; ++k) rows += d.T[k];
            for (int64_t sl = d.slot_base; sl < d.slot_base + rows * kWave; ++sl)
                out.slot_src[(size_t)sl] = (uint32_t)sl;
            for (int64_t li = (int64_t)d.tile0 * kWave; li < (int64_t)(d.tile0 + d.T[0]) * kWave; ++li)
                out.center_src[(size_t)li] = (uint32_t)(out.center_base + li);
        }
    }
    auto set_next = [&](int64_t station, int64_t next) {
        if (station < out.center_base) out.slot_next[(size_t)station] = (uint32_t)next;
        else if (station < out.tail_base)
            out.center_next[(size_t)(station - out.center_base)] = (uint32_t)next;
        else out.tail_next[(size_t)(station - out.tail_base)] = (uint32_t)next;
    };
    auto set_src = [&](int64_t station, int64_t from) {   // a pulled station's source
        if (station < out.center_base) out.slot_src[(size_t)station] = (uint32_t)from;
        else out.center_src[(size_t)(station - out.center_base)] = (uint32_t)from;
    };
    out.home.assign((size_t)n, kNoStation);
    parallel_nodes(n, 2 * m, [&](int32_t v0, int32_t v1) {
        std::vector<std::pair<int64_t, bool>> seq;   // (station, pulled)
        for (int32_t v = v0; v < v1; ++v) {
            seq.clear();
            const int64_t b = off[(size_t)v + 1];
            for (int64_t j = off[(size_t)v]; j < b;) {
                const int32_t p = ph[(size_t)j];
                int64_t k = j + 1;
                while (k < b && ph[(size_t)k] == p) ++k;
                if (p < P0)
                    seq.emplace_back(cen[(size_t)j] ? (int64_t)lane_station[(size_t)j]
                                                    : out.edge_slot[(size_t)at[(size_t)j]],
                                     pulled[(size_t)p] != 0);
                j = k;
            }
            if (local[(size_t)v] >= 0) seq.emplace_back(out.tail_base + local[(size_t)v], false);
            const size_t k = seq.size();
            if (k == 0) continue;
            for (size_t i = 0; i < k; ++i) {
                const auto &nx = seq[(i + 1) % k];
                set_next(seq[i].first, nx.second ? seq[i].first : nx.first);
                if (seq[i].second) set_src(seq[i].first, seq[(i + k - 1) % k].first);
            }
            // where the load rests between sweeps: what the first station reads
            out.home[(size_t)v] = (uint32_t)(seq[0].second ? seq[k - 1].first : seq[0].first);
        }
    });
    int64_t entries = out.tail_base + ntail_nodes;
    for (int32_t v = 0; v < n; ++v)
        if (out.home[(size_t)v] == kNoStation) out.home[(size_t)v] = (uint32_t)entries++;
    // one more entry, the sink: stores of padding rows and empty lanes go
    // there, so the kernels store without a branch
    if (entries + 1 >= (int64_t)kNoStation)
        fail(LOWD_E_UNSUPPORTED, "graph too large for 31-bit station indices");
    for (PhaseDescWide &d : out.desc) d.sink = (int32_t)entries;
    out.entries = entries + 1;
    // every index a pulled phase gathers at lies in the entry array
    for (const uint32_t x : out.slot_src)
        if ((int64_t)x >= out.entries) fail(LOWD_E_HIP, "pull source out of range");
    for (const uint32_t x : out.center_src)
        if ((int64_t)x >= out.entries) fail(LOWD_E_HIP, "pull source out of range");
    // the orientation bit rides on the leaf slot's next station
    parallel_chunks(P0 < P ? out.desc[(size_t)P0].slot_base : nslots, [&](int, int64_t lo, int64_t hi) {
        for (int64_t sl = lo; sl < hi; ++sl)
            if (out.slot_next[(size_t)sl] != kNoStation)
                out.slot_next[(size_t)sl] |= out.slot_leaf[(size_t)sl] & kCenterIsDst;
    });
}

}  // namespace lowd
