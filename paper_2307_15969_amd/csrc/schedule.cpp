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
#include <cmath>
#include <memory>
#include <numeric>
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

// Per-phase cost model (microseconds) used to place the split P0.  A phase
// run by a whole-GPU launch costs one kernel boundary inside a HIP graph plus
// its streamed bytes; a phase inside the LDS-resident workgroup costs a
// barrier plus its longest star chain plus one CU's streaming time.
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

// Edge indices 0..m-1 in ascending (visit_key, index) order: a stable LSD
// radix sort on the 64-bit keys (11-bit digits), so equal keys keep
// ascending index.
std::vector<int64_t> sort_by_visit_key(int64_t m) {
    std::vector<uint64_t> key((size_t)m), key2((size_t)m);
    std::vector<int64_t> idx((size_t)m), idx2((size_t)m);
    for (int64_t e = 0; e < m; ++e) {
        key[(size_t)e] = visit_key(e);
        idx[(size_t)e] = e;
    }
    constexpr int kDigit = 11;
    constexpr size_t kBuckets = (size_t)1 << kDigit;
    std::vector<int64_t> cnt(kBuckets);
    for (int shift = 0; shift < 64; shift += kDigit) {
        std::fill(cnt.begin(), cnt.end(), 0);
        for (int64_t i = 0; i < m; ++i) ++cnt[(size_t)(key[(size_t)i] >> shift) & (kBuckets - 1)];
        int64_t sum = 0;
        for (size_t b = 0; b < kBuckets; ++b) {
            const int64_t c = cnt[b];
            cnt[b] = sum;
            sum += c;
        }
        for (int64_t i = 0; i < m; ++i) {
            const size_t b = (size_t)(key[(size_t)i] >> shift) & (kBuckets - 1);
            const int64_t at = cnt[b]++;
            key2[(size_t)at] = key[(size_t)i];
            idx2[(size_t)at] = idx[(size_t)i];
        }
        key.swap(key2);
        idx.swap(idx2);
    }
    return idx;
}

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
                    Schedule &out, bool whole_in_lds) {
    out = Schedule();
    if (smax > kMaxStar && force_p0 != -2) {
        // the device layout holds stars of up to kMaxStar leaves; callers that
        // only want the phase assignment pass force_p0 = -2
        fail(LOWD_E_ARG, "star_max must be at most 32 for the sweep kernels");
    }
    out.n = n;
    out.m = m;
    out.smax = smax;
    out.phase.assign((size_t)m, 0);
    out.center.assign((size_t)m, 0);

    std::vector<int64_t> deg((size_t)n, 0);
    for (int64_t e = 0; e < m; ++e) {
        ++deg[(size_t)src[e]];
        ++deg[(size_t)dst[e]];
    }

    // ---- first fit --------------------------------------------------------
    // used[u]: phases where u has any role; noc[u]: phases where u cannot be
    // a center (it is a leaf there, or its star is full).
    // orientation, visiting order (ascending (key, index))
    std::vector<int32_t> ctr((size_t)m), lf((size_t)m);
    for (int64_t e = 0; e < m; ++e) {
        const int32_t a = src[e], b = dst[e];
        if (deg[(size_t)a] > deg[(size_t)b] || (deg[(size_t)a] == deg[(size_t)b] && a < b)) {
            ctr[(size_t)e] = a;
            lf[(size_t)e] = b;
        } else {
            ctr[(size_t)e] = b;
            lf[(size_t)e] = a;
        }
    }
    const std::vector<int64_t> visit = sort_by_visit_key(m);
    // the edges' centers and leaves in visiting order: the loop below then
    // streams through them and can prefetch the node state ahead
    std::vector<int32_t> cv((size_t)m), lv((size_t)m);
    for (int64_t i = 0; i < m; ++i) {
        cv[(size_t)i] = ctr[(size_t)visit[(size_t)i]];
        lv[(size_t)i] = lf[(size_t)visit[(size_t)i]];
    }
    std::vector<int32_t> pv((size_t)m);
    // The first 64 phases of every node live in flat arrays (one word per
    // node, one byte per (node, phase) for star sizes); later phases, which
    // only high-degree nodes reach, in per-node overflow storage.  The
    // visiting order touches nodes at random, so the next edges' node state
    // is prefetched.
    std::vector<uint64_t> used0((size_t)n, 0), noc0((size_t)n, 0);
    std::vector<uint8_t> cnt0((size_t)n * 64, 0);
    struct Overflow {
        Bits used, noc;
        std::vector<uint8_t> cnt;   // star sizes of phases 64, 65, ...
    };
    std::vector<std::unique_ptr<Overflow>> ov((size_t)n);
    auto used_word = [&](int32_t u, size_t wi) -> uint64_t {
        if (wi == 0) return used0[(size_t)u];
        const Overflow *o = ov[(size_t)u].get();
        return o ? o->used.word(wi - 1) : 0ull;
    };
    auto noc_word = [&](int32_t u, size_t wi) -> uint64_t {
        if (wi == 0) return noc0[(size_t)u];
        const Overflow *o = ov[(size_t)u].get();
        return o ? o->noc.word(wi - 1) : 0ull;
    };
    auto over = [&](int32_t u) -> Overflow & {
        if (!ov[(size_t)u]) ov[(size_t)u].reset(new Overflow());
        return *ov[(size_t)u];
    };
    constexpr int64_t kAhead = 8;
    int32_t P = 0;
    for (int64_t i = 0; i < m; ++i) {
        if (i + kAhead < m) {
            const int32_t ca = cv[(size_t)(i + kAhead)], la = lv[(size_t)(i + kAhead)];
            __builtin_prefetch(&noc0[(size_t)ca]);
            __builtin_prefetch(&used0[(size_t)ca]);
            __builtin_prefetch(&used0[(size_t)la]);
            __builtin_prefetch(&noc0[(size_t)la]);
            __builtin_prefetch(&cnt0[(size_t)ca * 64]);
        }
        const int32_t c = cv[(size_t)i], l = lv[(size_t)i];
        int32_t p = 0;
        for (size_t wi = 0;; ++wi) {
            const uint64_t busy = noc_word(c, wi) | used_word(l, wi);
            if (~busy) {
                p = (int32_t)(wi * 64 + (size_t)__builtin_ctzll(~busy));
                break;
            }
        }
        uint8_t *cc;
        if (p < 64) {
            const uint64_t bit = 1ull << p;
            used0[(size_t)c] |= bit;
            used0[(size_t)l] |= bit;
            noc0[(size_t)l] |= bit;
            cc = &cnt0[(size_t)c * 64 + (size_t)p];
            if (++*cc >= smax) noc0[(size_t)c] |= bit;
        } else {
            const int32_t q = p - 64;
            Overflow &oc = over(c);
            oc.used.set(q);
            Overflow &ol = over(l);
            ol.used.set(q);
            ol.noc.set(q);
            if ((size_t)q >= oc.cnt.size()) oc.cnt.resize((size_t)q + 1 + ((size_t)q >> 1), 0);
            if (++oc.cnt[(size_t)q] >= smax) oc.noc.set(q);
        }
        pv[(size_t)i] = p;
        if (p + 1 > P) P = p + 1;
    }
    out.P = P;
    for (int64_t i = 0; i < m; ++i) out.phase[(size_t)visit[(size_t)i]] = pv[(size_t)i];
    out.center = std::move(ctr);
    std::vector<uint64_t>().swap(used0);
    std::vector<uint64_t>().swap(noc0);
    std::vector<uint8_t>().swap(cnt0);
    std::vector<std::unique_ptr<Overflow>>().swap(ov);

    if (force_p0 == -2) return;   // phase assignment only

    // ---- edges by (phase, center, index) -----------------------------------
    std::vector<int64_t> pstart((size_t)P + 1, 0);
    for (int64_t e = 0; e < m; ++e) ++pstart[(size_t)out.phase[(size_t)e] + 1];
    for (int32_t p = 0; p < P; ++p) pstart[(size_t)p + 1] += pstart[(size_t)p];
    // two stable counting sorts: by center, then by phase, so a phase's
    // edges come grouped by center (ascending) in ascending edge index
    std::vector<int64_t> byphase((size_t)m);
    {
        std::vector<int64_t> cstart((size_t)n + 1, 0);
        for (int64_t e = 0; e < m; ++e) ++cstart[(size_t)out.center[(size_t)e] + 1];
        for (int32_t u = 0; u < n; ++u) cstart[(size_t)u + 1] += cstart[(size_t)u];
        std::vector<int64_t> bycenter((size_t)m);
        for (int64_t e = 0; e < m; ++e) bycenter[(size_t)cstart[(size_t)out.center[(size_t)e]]++] = e;
        std::vector<int64_t> cur(pstart.begin(), pstart.end() - 1);
        for (int64_t i = 0; i < m; ++i) {
            const int64_t e = bycenter[(size_t)i];
            byphase[(size_t)cur[(size_t)out.phase[(size_t)e]]++] = e;
        }
    }
    std::vector<int64_t> ecount((size_t)P, 0), maxstar((size_t)P, 0);
    // stars per phase: (begin, len) into byphase
    struct Star { int64_t begin; int32_t len; int32_t center; };
    std::vector<std::vector<Star>> stars((size_t)P);
    for (int32_t p = 0; p < P; ++p) {
        ecount[(size_t)p] = pstart[(size_t)p + 1] - pstart[(size_t)p];
        std::vector<Star> &st = stars[(size_t)p];
        for (int64_t i = pstart[(size_t)p]; i < pstart[(size_t)p + 1];) {
            int32_t c = out.center[(size_t)byphase[(size_t)i]];
            int64_t j = i;
            while (j < pstart[(size_t)p + 1] && out.center[(size_t)byphase[(size_t)j]] == c) ++j;
            st.push_back(Star{i, (int32_t)(j - i), c});
            maxstar[(size_t)p] = std::max<int64_t>(maxstar[(size_t)p], j - i);
            i = j;
        }
        std::sort(st.begin(), st.end(), [](const Star &x, const Star &y) {
            return x.len != y.len ? x.len > y.len : x.center < y.center;
        });
    }

    // ---- split P0 ---------------------------------------------------------
    std::vector<int32_t> last((size_t)n, -1);
    for (int64_t e = 0; e < m; ++e) {
        int32_t p = out.phase[(size_t)e];
        last[(size_t)src[e]] = std::max(last[(size_t)src[e]], p);
        last[(size_t)dst[e]] = std::max(last[(size_t)dst[e]], p);
    }
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
        if ((int64_t)stars[(size_t)p].size() > (int64_t)kTailWaves * kWave) min_p0 = p + 1;
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
        const double tiles = (double)((stars[(size_t)p].size() + kWave - 1) / kWave);
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
    int64_t ntiles = 0, nslots = 0;
    for (int32_t p = 0; p < P; ++p) {
        const std::vector<Star> &st = stars[(size_t)p];
        PhaseDescWide &d = out.desc[(size_t)p];
        d.slot_base = nslots;
        d.tile0 = (int32_t)ntiles;
        d.sink = 0;
        int32_t t = (int32_t)((st.size() + kWave - 1) / kWave);
        for (int k = 0; k < kMaxStar; ++k) {
            int32_t cnt = 0;   // tiles whose first (deepest) star is longer than k
            for (int32_t i = 0; i < t; ++i)
                if (st[(size_t)i * kWave].len > k) ++cnt;
            d.T[k] = cnt;
            nslots += (int64_t)cnt * kWave;
        }
        out.phase_depth[(size_t)p] = st.empty() ? 0 : st[0].len;
        ntiles += t;
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
    std::vector<int64_t> first((size_t)n, -1), prev((size_t)n, -1);
    auto set_next = [&](int64_t station, int64_t next) {
        if (station < out.center_base) out.slot_next[(size_t)station] = (uint32_t)next;
        else if (station < out.tail_base)
            out.center_next[(size_t)(station - out.center_base)] = (uint32_t)next;
        else out.tail_next[(size_t)(station - out.tail_base)] = (uint32_t)next;
    };
    auto arrive = [&](int32_t v, int64_t station) {
        if (prev[(size_t)v] < 0) first[(size_t)v] = station;
        else set_next(prev[(size_t)v], station);
        prev[(size_t)v] = station;
    };
    for (int32_t p = 0; p < P; ++p) {
        const bool tail = p >= P0;
        if (tail) out.tail_edges += ecount[(size_t)p];
        if (tail) {
            // tail dummies are the LDS entries after the tail's nodes
            const int64_t t = (int64_t)((stars[(size_t)p].size() + kWave - 1) / kWave);
            for (int64_t i = 0; i < t * kWave; ++i)
                out.tile_center[(size_t)(out.desc[(size_t)p].tile0 * kWave + i)] = ntail_nodes;
            const PhaseDescWide &dd = out.desc[(size_t)p];
            int64_t rows = 0;
            for (int k = 0; k < kMaxStar; ++k) rows += dd.T[k];
            for (int64_t i = 0; i < rows * kWave; ++i)
                out.slot_leaf[(size_t)(dd.slot_base + i)] = (uint32_t)ntail_nodes + 1u;
        }
        const std::vector<Star> &st = stars[(size_t)p];
        const PhaseDescWide &d = out.desc[(size_t)p];
        for (size_t i = 0; i < st.size(); ++i) {
            const Star &sr = st[i];
            const int64_t tt = (int64_t)(i / kWave);
            const int lane = (int)(i % kWave);
            int64_t rows_before = 0;   // sum_k min(T[k], tt)
            for (int k = 0; k < kMaxStar; ++k) rows_before += std::min<int64_t>(d.T[k], tt);
            const int64_t tile_base = d.slot_base + rows_before * kWave;
            out.tile_center[(size_t)((d.tile0 + tt) * kWave + lane)] =
                tail ? local[(size_t)sr.center] : sr.center;
            if (!tail) arrive(sr.center, out.center_base + (d.tile0 + tt) * kWave + lane);
            for (int32_t k = 0; k < sr.len; ++k) {
                int64_t e = byphase[(size_t)(sr.begin + k)];
                bool c_is_dst = dst[e] == sr.center;
                int32_t leaf = c_is_dst ? src[e] : dst[e];
                int32_t id = tail ? local[(size_t)leaf] : leaf;
                int64_t sl = tile_base + (int64_t)k * kWave + lane;
                out.slot_leaf[(size_t)sl] = (uint32_t)id | (c_is_dst ? kCenterIsDst : 0u);
                out.slot_edge[(size_t)sl] = e;
                out.edge_slot[(size_t)e] = sl;
                if (!tail) arrive(leaf, sl);
            }
        }
    }
    for (int32_t j = 0; j < ntail_nodes; ++j) arrive(out.tail_nodes[(size_t)j], out.tail_base + j);
    // close each node's cycle; nodes on no edge get a home entry of their own
    int64_t entries = out.tail_base + ntail_nodes;
    out.home.assign((size_t)n, kNoStation);
    for (int32_t v = 0; v < n; ++v) {
        if (prev[(size_t)v] >= 0) set_next(prev[(size_t)v], first[(size_t)v]);
        else first[(size_t)v] = entries++;
        out.home[(size_t)v] = (uint32_t)first[(size_t)v];
    }
    // one more entry, the sink: stores of padding rows and empty lanes go
    // there, so the kernels store without a branch
    if (entries + 1 >= (int64_t)kNoStation)
        fail(LOWD_E_UNSUPPORTED, "graph too large for 31-bit station indices");
    for (PhaseDescWide &d : out.desc) d.sink = (int32_t)entries;
    out.entries = entries + 1;
    // the orientation bit rides on the leaf slot's next station
    for (int64_t sl = 0; sl < (P0 < P ? out.desc[(size_t)P0].slot_base : nslots); ++sl)
        if (out.slot_next[(size_t)sl] != kNoStation)
            out.slot_next[(size_t)sl] |= out.slot_leaf[(size_t)sl] & kCenterIsDst;
}

}  // namespace lowd
