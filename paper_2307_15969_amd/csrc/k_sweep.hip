// k_sweep.hip -- initialisation, the LOWD edge sweep and its convergence
// statistics.
//
// The sweep follows the phase schedule (schedule.cpp): one kernel per phase
// for the wide phases, then narrower phases inside one workgroup, and the
// narrow last phases inside one workgroup that keeps their nodes' loads in
// LDS.  Inside a phase every lane owns one star: it keeps the center's load
// in a register, and walks the star's leaves in order, applying Algorithm
// 1's locally optimal step to each edge.  The stars of a phase share no
// node, so no atomics are needed and the result is that of the sequential
// edge loop in schedule order.
//
// Outside the LDS tier a node's load lives at its next station (see the
// schedule): a phase reads the loads of its leaves and centers in slot
// order, together with the fractions, and writes every updated load to the
// node's next station, so no read of a phase waits for an address.
#include "lowd_internal.h"
#include "sweep_state.h"
#include "wg_check.h"

namespace lowd {
namespace {

// ------------------------------------------------------------ init ------
template <class St, bool kWeighted>
__global__ void k_init_slots(int64_t nslots, const int64_t *slot_edge, const float *w,
                             typename St::X *slot_x, float *slot_w) {
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < nslots;
         s += (int64_t)gridDim.x * blockDim.x) {
        int64_t e = slot_edge[s];
        float we = (kWeighted && e >= 0) ? w[e] : 1.0f;
        // a padding slot holds its whole weight (1): its step is a no-op
        slot_x[s] = e >= 0 ? St::half_weight(we) : (typename St::X)1.0f;
        if (kWeighted) slot_w[s] = we;
    }
}

// Station entries before any load is placed: slot entries +infinity (the
// load a padding row reads: its step is then a no-op), lane entries and the
// rest zero (the center of a lane without a star).  Non-station entries keep
// these values: no station names them as next.
template <class St>
__global__ void k_fill_entries(int64_t entries, int64_t center_base, typename St::L *E) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < entries;
         i += (int64_t)gridDim.x * blockDim.x)
        E[i] = i < center_base ? St::infinite() : St::from_f64(0.0);
}

// l_u = sum of w_e / 2 over the edges at u, in ascending edge index, placed
// at u's first station.  Weighted rows of kBigRow entries or more are left to
// k_init_loads_big.
template <class St, bool kWeighted>
__global__ void k_init_loads(int32_t n, const int64_t *row_ptr, const uint32_t *inc,
                             const float *w, const uint32_t *home, typename St::L *E) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        if (kWeighted) {
            if (row_ptr[u + 1] - row_ptr[u] >= kBigRow) continue;
            for (int64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j)
                acc = acc + (double)w[inc[j] >> 1] / 2.0;
        } else {
            // a sum of halves is exact in any order: deg / 2
            acc = (double)(row_ptr[u + 1] - row_ptr[u]) * 0.5;
        }
        E[home[u]] = St::from_f64(acc);
    }
}

// The same ascending-order sum for one long weighted row per wave: the wave
// loads 64 consecutive halves at a time and every lane adds them in order
// (lanes past the row's end contribute +0, which leaves a sum of
// non-negative terms unchanged), so the bits equal the sequential sum.
template <class St>
__global__ void __launch_bounds__(kWave) k_init_loads_big(const int32_t *big,
                                                          const int64_t *row_ptr,
                                                          const uint32_t *inc, const float *w,
                                                          const uint32_t *home,
                                                          typename St::L *E) {
    const int32_t u = big[blockIdx.x];
    const int lane = threadIdx.x;
    const int64_t end = row_ptr[u + 1];
    double acc = 0.0;
    for (int64_t j0 = row_ptr[u]; j0 < end; j0 += kWave) {
        const int64_t j = j0 + lane;
        const double h = j < end ? (double)w[inc[j] >> 1] / 2.0 : 0.0;
        const uint64_t hb = __builtin_bit_cast(uint64_t, h);
        const uint32_t lo = (uint32_t)hb, hi = (uint32_t)(hb >> 32);
#pragma unroll
        for (int k = 0; k < kWave; ++k) {
            const uint64_t v = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(hi, k) << 32) |
                               (uint32_t)__builtin_amdgcn_readlane(lo, k);
            acc = acc + __builtin_bit_cast(double, v);
        }
    }
    if (lane == 0) E[home[u]] = St::from_f64(acc);
}

// ------------------------------------------------------------ one tile ---
// One wave = one tile of 64 stars of a phase; the lane's star has a center c
// and depth leaves in rows 0..depth-1 of the tile.  A tile is loaded in one
// go (center, leaf ids, fractions, weights: every address follows from the
// phase descriptor), then the endpoint loads are read together, then the
// lane runs its chain of depth steps in registers, carrying the center's
// load.  Leaves of one star are distinct and belong to no other star of the
// phase, so all reads of a tile can be in flight at once.
template <class St, bool kWeighted>
struct Tile {
    int32_t c;
    int32_t depth;        // wave-uniform
    int64_t base;         // wave-uniform: first slot of the tile
    uint32_t enc[kTierStar];
    typename St::X x[kTierStar];
    float w[kTierStar];
};

template <class St, bool kWeighted>
__device__ __forceinline__ void load_tile(Tile<St, kWeighted> &tl, const PhaseDesc &d, int32_t t,
                                          int lane, const int32_t *__restrict__ tile_center,
                                          const uint32_t *__restrict__ slot_leaf,
                                          const typename St::X *__restrict__ slot_x,
                                          const float *__restrict__ slot_w) {
    int32_t depth = 0;
    int64_t rows = 0;
#pragma unroll
    for (int k = 0; k < kTierStar; ++k) {
        depth += (d.T[k] > t) ? 1 : 0;
        rows += (int64_t)(d.T[k] < t ? d.T[k] : t);
    }
    tl.depth = __builtin_amdgcn_readfirstlane(depth);
    const int64_t base = d.slot_base + rows * kWave;
    tl.base = base;
    tl.c = tile_center[(int64_t)(d.tile0 + t) * kWave + lane];
    const uint32_t *pl = slot_leaf + base + lane;
    const typename St::X *px = slot_x + base + lane;
    const float *pw = kWeighted ? slot_w + base + lane : nullptr;
    if (tl.depth == kTierStar) {   // a full tile: no per-row guard
#pragma unroll
        for (int k = 0; k < kTierStar; ++k) {
            tl.enc[k] = pl[k * kWave];
            tl.x[k] = px[k * kWave];
            tl.w[k] = kWeighted ? pw[k * kWave] : 1.0f;
        }
        return;
    }
#pragma unroll
    for (int k = 0; k < kTierStar; ++k) {
        if (k < tl.depth) {
            tl.enc[k] = pl[k * kWave];
            tl.x[k] = px[k * kWave];
            tl.w[k] = kWeighted ? pw[k * kWave] : 1.0f;
        }
    }
}

// Branch-free per lane.  A padding row (the lane's star is shorter than the
// tile) names the "infinite" dummy leaf with fraction equal to its weight:
// there the step moves d = min(inf, 0) = 0, an exact no-op for the center.
// A lane without a star has the zero dummy as its center and only padding.
template <class St, bool kWeighted, class LPtr>
__device__ __forceinline__ void run_tile(Tile<St, kWeighted> &tl, int lane,
                                         typename St::X *__restrict__ slot_x, LPtr L) {
    using T = typename std::remove_cv<typename std::remove_reference<decltype(L[0])>::type>::type;
    const T lc_raw = L[tl.c];
    T raw[kTierStar];
    typename St::R Ll[kTierStar];
    typename St::X *px = slot_x + tl.base + lane;
    if (tl.depth == kTierStar) {   // a full tile: one straight block
#pragma unroll
        for (int k = 0; k < kTierStar; ++k) raw[k] = L[tl.enc[k] & ~kCenterIsDst];
        typename St::R Lc = widen(lc_raw);
#pragma unroll
        for (int k = 0; k < kTierStar; ++k) Ll[k] = widen(raw[k]);
#pragma unroll
        for (int k = 0; k < kTierStar; ++k)
            St::step_center(Lc, Ll[k], tl.enc[k] & kCenterIsDst, tl.x[k], tl.w[k]);
#pragma unroll
        for (int k = 0; k < kTierStar; ++k) {
            px[k * kWave] = tl.x[k];
            L[tl.enc[k] & ~kCenterIsDst] = narrow<T>(Ll[k]);
        }
        L[tl.c] = narrow<T>(Lc);
        return;
    }
#pragma unroll
    for (int k = 0; k < kTierStar; ++k) {
        if (k < tl.depth) raw[k] = L[tl.enc[k] & ~kCenterIsDst];
        else raw[k] = narrow<T>(__builtin_inf());
    }
    // widened after all the loads are issued (a conversion next to a guarded
    // load makes the compiler wait for that load before issuing the next)
    typename St::R Lc = widen(lc_raw);
#pragma unroll
    for (int k = 0; k < kTierStar; ++k) Ll[k] = widen(raw[k]);
#pragma unroll
    for (int k = 0; k < kTierStar; ++k)
        if (k < tl.depth) St::step_center(Lc, Ll[k], tl.enc[k] & kCenterIsDst, tl.x[k], tl.w[k]);
#pragma unroll
    for (int k = 0; k < kTierStar; ++k) {
        if (k < tl.depth) {
            px[k * kWave] = tl.x[k];
            L[tl.enc[k] & ~kCenterIsDst] = narrow<T>(Ll[k]);
        }
    }
    L[tl.c] = narrow<T>(Lc);
}

// ---------------------------------------------- one tile, station form --
// The same tile for the phases outside the LDS tier: besides the fractions
// the lane reads its center's load (the lane's own station entry) and its
// leaves' loads (the slots' station entries) in slot order, plus where each
// goes next.  Padding rows read +infinity and lanes without a star read a
// zero center; neither is written back.
template <class St, bool kWeighted, int D>
struct StationTile {
    int32_t depth;        // wave-uniform
    int64_t base;         // wave-uniform: first slot of the tile
    int64_t lane_entry;   // the lane's center station
    uint32_t cnext;       // next station of the center, or the sink
    uint32_t sink;
    uint32_t nx[D];
    typename St::X x[D];
    float w[D];
    typename St::L lc_raw;             // the loads as stored, widened after the
    typename St::L ll_raw[D];   // tile's single wait (see run_station_tile)
    typename St::R lc;
    typename St::R ll[D];
};

// A tile's depth and first slot.  Tile t of a phase has depth
// #{k : T[k] > t} and follows sum_k min(T[k], t) full rows of the phase.
template <int D>
__device__ __forceinline__ void tile_geometry(const PhaseDescT<D> &d, int32_t t, int32_t &depth,
                                              int64_t &base) {
    int32_t dp = 0;
    int64_t rows = 0;
#pragma unroll
    for (int k = 0; k < D; ++k) {
        dp += (d.T[k] > t) ? 1 : 0;
        rows += (int64_t)(d.T[k] < t ? d.T[k] : t);
    }
    depth = __builtin_amdgcn_readfirstlane(dp);
    base = d.slot_base + rows * kWave;
}

// the parts that do not depend on the previous phase, for a tile of the
// given depth whose rows start at slot `base`; li = the lane's index among
// all tile lanes
template <class St, bool kWeighted, int D>
__device__ __forceinline__ void load_static_at(StationTile<St, kWeighted, D> &tl, int32_t depth,
                                               int64_t base, int64_t li, int lane,
                                               int64_t center_base,
                                               const uint32_t *__restrict__ center_next,
                                               const uint32_t *__restrict__ slot_next,
                                               const typename St::X *__restrict__ slot_x,
                                               const float *__restrict__ slot_w) {
    tl.depth = depth;
    tl.base = base;
    tl.lane_entry = center_base + li;
    const uint32_t *pn = slot_next + base + lane;
    const typename St::X *px = slot_x + base + lane;
    const float *pw = kWeighted ? slot_w + base + lane : nullptr;
    if (tl.depth == D) {   // a full tile: no per-row guard
#pragma unroll
        for (int k = 0; k < D; ++k) {
            tl.nx[k] = pn[k * kWave];
            tl.x[k] = px[k * kWave];
            tl.w[k] = kWeighted ? pw[k * kWave] : 1.0f;
        }
    } else {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            if (k < tl.depth) {
                tl.nx[k] = pn[k * kWave];
                tl.x[k] = px[k * kWave];
                tl.w[k] = kWeighted ? pw[k * kWave] : 1.0f;
            }
        }
    }
    // last: in k_phase center_next is the first argument not preloaded
    tl.cnext = center_next[li];
}

template <class St, bool kWeighted, int D>
__device__ __forceinline__ void load_static(StationTile<St, kWeighted, D> &tl, const PhaseDescT<D> &d,
                                            int32_t t, int lane, int64_t center_base,
                                            const uint32_t *__restrict__ center_next,
                                            const uint32_t *__restrict__ slot_next,
                                            const typename St::X *__restrict__ slot_x,
                                            const float *__restrict__ slot_w) {
    int32_t depth;
    int64_t base;
    tile_geometry(d, t, depth, base);
    load_static_at(tl, depth, base, (int64_t)(d.tile0 + t) * kWave + lane, lane, center_base,
                   center_next, slot_next, slot_x, slot_w);
    tl.sink = (uint32_t)d.sink;
}

// the loads of a pulled phase, gathered from each node's previous station
// (the rows' and the lane's source entries first, in one batch)
template <class St, bool kWeighted, int D>
__device__ __forceinline__ void pull_loads(StationTile<St, kWeighted, D> &tl, int lane,
                                           int64_t li, const typename St::L *E,
                                           const uint32_t *__restrict__ slot_src,
                                           const uint32_t *__restrict__ center_src) {
    uint32_t from[D];
    const uint32_t *ps = slot_src + tl.base + lane;
    const uint32_t cfrom = center_src[li];
    if (tl.depth == D) {
#pragma unroll
        for (int k = 0; k < D; ++k) from[k] = ps[k * kWave];
    } else {
#pragma unroll
        for (int k = 0; k < D; ++k) from[k] = k < tl.depth ? ps[k * kWave] : 0u;
    }
    tl.lc_raw = E[cfrom];
    if (tl.depth == D) {
#pragma unroll
        for (int k = 0; k < D; ++k) tl.ll_raw[k] = E[from[k]];
        return;
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
        if (k < tl.depth) tl.ll_raw[k] = E[from[k]];
        else tl.ll_raw[k] = St::infinite();
    }
}

// the loads, written by earlier phases
template <class St, bool kWeighted, int D>
__device__ __forceinline__ void load_loads(StationTile<St, kWeighted, D> &tl, int lane,
                                           const typename St::L *E) {
    tl.lc_raw = E[tl.lane_entry];
    const typename St::L *pl = E + tl.base + lane;
    if (tl.depth == D) {
#pragma unroll
        for (int k = 0; k < D; ++k) tl.ll_raw[k] = pl[k * kWave];
        return;
    }
#pragma unroll
    for (int k = 0; k < D; ++k) {
        if (k < tl.depth) tl.ll_raw[k] = pl[k * kWave];
        else tl.ll_raw[k] = St::infinite();
    }
}

// A row without a next station (padding, or a lane without a star) stores
// into the sink entry, so the stores need no per-lane branch; a full tile
// needs no per-row guard either, and its rows form one straight block.
template <class St, bool kWeighted, int D>
__device__ __forceinline__ void run_station_tile(StationTile<St, kWeighted, D> &tl, int lane,
                                                 typename St::X *__restrict__ slot_x,
                                                 typename St::L *E) {
    typename St::X *px = slot_x + tl.base + lane;
    // widen the loads here, after the wait: a conversion next to a guarded
    // load makes the compiler wait for each load before issuing the next
    tl.lc = St::to_f64(tl.lc_raw);
#pragma unroll
    for (int k = 0; k < D; ++k) tl.ll[k] = St::to_f64(tl.ll_raw[k]);
    // A leaf's load and the edge's fraction are final after its step: their
    // stores go out right behind it, while the chain's next steps (which
    // depend only on the center's load) run, instead of after the chain.
    if (tl.depth == D) {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            St::step_center(tl.lc, tl.ll[k], tl.nx[k] & kCenterIsDst, tl.x[k], tl.w[k]);
            px[k * kWave] = tl.x[k];
            const uint32_t nx = tl.nx[k] & ~kCenterIsDst;
            E[nx != kNoStation ? nx : tl.sink] = St::from_f64(tl.ll[k]);
        }
    } else {
#pragma unroll
        for (int k = 0; k < D; ++k) {
            if (k < tl.depth) {
                St::step_center(tl.lc, tl.ll[k], tl.nx[k] & kCenterIsDst, tl.x[k], tl.w[k]);
                px[k * kWave] = tl.x[k];
                const uint32_t nx = tl.nx[k] & ~kCenterIsDst;
                E[nx != kNoStation ? nx : tl.sink] = St::from_f64(tl.ll[k]);
            }
        }
    }
    E[tl.cnext != kNoStation ? tl.cnext : tl.sink] = St::from_f64(tl.lc);
}

// --------------------------------------------------- whole-GPU phase -----
// One wave per block.  A narrow phase (few tiles) would leave most CUs idle
// while each busy CU works through up to 16 x 64 random load and store
// lines of its tile, bounded by the misses one CU keeps in flight; such a
// phase is spread instead: a tile is shared by 2^spread waves, each running
// 64 >> spread of its lanes (lanes outside the wave's share exit at once).
constexpr int kPhaseBlock = 64;
// s_waitcnt immediate: vector memory count 0, the other counters not waited
constexpr int kWaitLoads = 0x0F70;
static_assert(kWave == 64, "lane shares assume 64-wide waves");
constexpr int kMaxSpreadLog2 = 3;    // at least 8 lanes per wave
constexpr int32_t kSpreadWaves = 256;  // spread until about one wave per CU

// The first 16 dwords of the arguments (through center_next) are all a full
// tile needs before its first loads; they are preloaded into scalar
// registers at wave launch, so a full tile's loads do not wait for the
// argument fetch (the descriptor and slot_w follow).  full_tiles = T[D-1]:
// tiles t < full_tiles have depth D and start at slot_base + D * 64 * t.
// D = 16 for phases whose stars have at most 16 leaves, 32 for deeper ones
// (a lane then keeps 32 leaves' fractions and loads in registers).  kPull:
// a pulled phase, whose loads are gathered through slot_src / center_src
// (one more dependent round trip; its writes are coalesced instead of
// scattered, see Schedule).
template <class St, bool kWeighted, int D, bool kPull>
__global__ void __launch_bounds__(kPhaseBlock)
k_phase(int64_t slot_base, int32_t tile0, int32_t tiles, int32_t full_tiles, int32_t spread,
        int64_t center_base, typename St::L *__restrict__ E,
        const uint32_t *__restrict__ slot_next, typename St::X *__restrict__ slot_x,
        const uint32_t *__restrict__ center_next, PhaseDescT<D> d,
        const float *__restrict__ slot_w, const uint32_t *__restrict__ slot_src,
        const uint32_t *__restrict__ center_src) {
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t t = __builtin_amdgcn_readfirstlane((int32_t)(blockIdx.x >> spread));
    if (t >= tiles) return;
    const int32_t share = (int32_t)(blockIdx.x & ((1u << spread) - 1));
    if ((lane >> (6 - spread)) != share) return;
    int32_t depth = D;
    int64_t base = slot_base + (int64_t)t * (D * kWave);
    if (t >= full_tiles) tile_geometry(d, t, depth, base);
    StationTile<St, kWeighted, D> tl;
    const int64_t li = (int64_t)(tile0 + t) * kWave + lane;
    load_static_at(tl, depth, base, li, lane, center_base, center_next, slot_next, slot_x, slot_w);
    if (kPull) pull_loads(tl, lane, li, E, slot_src, center_src);
    else load_loads(tl, lane, E);
    tl.sink = (uint32_t)d.sink;
    // Every load of the tile is needed before the chain.  Waiting for all of
    // them here, on every path, keeps the compiler's per-path wait tracking
    // from placing a wait for the previous store before each store.
    __builtin_amdgcn_s_waitcnt(kWaitLoads);
    run_station_tile(tl, lane, slot_x, E);
}

// ------------------------------------------- whole-GPU phase, node form --
// For graphs whose phases are wide (millions of edges each), the loads live
// in one node-indexed array E[n + 2] (E[n] the zero center of empty lanes,
// E[n+1] the infinite leaf of padding rows) instead of at stations: it is
// small enough to stay in the on-die caches (the 256 MB Infinity Cache and
// the L2s), while the station array of such a graph is as large as its edge
// list and every scattered write to it goes to HBM.  A tile's leaf ids and
// fractions stream in coalesced; its loads are gathered by id, the chain
// runs as in k_phase, and each leaf's load is scattered back by id right
// behind its step.  Leaves of one phase are distinct and no center is a
// leaf, so no two lanes touch one entry.
template <class St, bool kWeighted, int D>
__global__ void __launch_bounds__(kPhaseBlock)
k_phase_node(PhaseDescT<D> d, int32_t spread, const int32_t *__restrict__ tile_center,
             const uint32_t *__restrict__ slot_leaf, typename St::X *__restrict__ slot_x,
             const float *__restrict__ slot_w, typename St::L *__restrict__ E) {
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t t = __builtin_amdgcn_readfirstlane((int32_t)(blockIdx.x >> spread));
    if (t >= d.T[0]) return;
    const int32_t share = (int32_t)(blockIdx.x & ((1u << spread) - 1));
    if ((lane >> (6 - spread)) != share) return;
    int32_t depth;
    int64_t base;
    tile_geometry(d, t, depth, base);
    const int32_t c = tile_center[(int64_t)(d.tile0 + t) * kWave + lane];
    const uint32_t *pl = slot_leaf + base + lane;
    typename St::X *px = slot_x + base + lane;
    const float *pw = kWeighted ? slot_w + base + lane : nullptr;
    uint32_t enc[D];
    typename St::X x[D];
    float w[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        if (k < depth) {
            enc[k] = pl[k * kWave];
            x[k] = px[k * kWave];
            w[k] = kWeighted ? pw[k * kWave] : 1.0f;
        } else {
            enc[k] = 0u;
        }
    }
    // the gathers, then one wait for all of them (see k_phase)
    const typename St::L lc_raw = E[c];
    typename St::L raw[D];
#pragma unroll
    for (int k = 0; k < D; ++k) {
        if (k < depth) raw[k] = E[enc[k] & ~kCenterIsDst];
        else raw[k] = St::infinite();
    }
    __builtin_amdgcn_s_waitcnt(kWaitLoads);
    typename St::R lc = St::to_f64(lc_raw);
    typename St::R ll[D];
#pragma unroll
    for (int k = 0; k < D; ++k) ll[k] = St::to_f64(raw[k]);
#pragma unroll
    for (int k = 0; k < D; ++k) {
        if (k < depth) {
            St::step_center(lc, ll[k], enc[k] & kCenterIsDst, x[k], w[k]);
            px[k * kWave] = x[k];
            E[enc[k] & ~kCenterIsDst] = St::from_f64(ll[k]);
        }
    }
    E[c] = St::from_f64(lc);
}

// initial node-form entries: every node and the zero center 0, the
// padding leaf +infinity (the initial loads follow, k_init_loads)
template <class St>
__global__ void k_fill_nodes(int32_t n, typename St::L *E) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < (int64_t)n + 2;
         i += (int64_t)gridDim.x * blockDim.x)
        E[i] = i == (int64_t)n + 1 ? St::infinite() : St::from_f64(0.0);
}

// ----------------------------------------- single-workgroup phases -------
// The narrow phases after the whole-GPU ones run inside ONE workgroup, one
// after another, separated by workgroup barriers instead of kernel
// boundaries:
//  * middle phases (k_mid): the loads stay at their stations in global
//    memory; all accesses come from one CU, so they are coherent through its
//    caches and a workgroup barrier orders them (one CU's memory rate bounds
//    this tier: it pays only for phases of a few hundred edges);
//  * last phases (k_tail): their nodes' loads are staged in LDS (with the
//    tail's own dummy entries) and written back to their next stations at
//    the end; an LDS-only barrier orders them.
// Wave w owns tiles w, w + W, ... of every phase.  Each wave keeps two tile
// buffers: while it runs phase p from one, the other already receives its
// first tile of phase p+1 (leaf ids, fractions and next stations do not
// depend on phase p; only the loads do).  The buffers alternate, so no
// register copy forces the prefetch to complete.  Phase descriptors are
// staged in LDS.
constexpr int kTailBlock = 512;
// lanes that share one node's incidence row in the per-node sums
constexpr int kRowLanes = 8;
static_assert(kTailBlock / kWave == kTailWaves, "tail width");

// Barrier that orders LDS only: every wave's LDS writes are complete before
// any wave passes.  Outstanding global loads (the next phase's prefetch) and
// stores (fractions, read again only in the next sweep) are not waited for.
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// The descriptor of phase p, read from LDS into one VGPR (lane i holds
// word i) and broadcast into scalar registers.
__device__ __forceinline__ PhaseDesc desc_from_lds(const PhaseDesc *sd, int32_t p, int lane) {
    constexpr int kWords = (int)(sizeof(PhaseDesc) / 4);
    const int32_t *w = reinterpret_cast<const int32_t *>(sd + p);
    const int32_t v = lane < kWords ? w[lane] : 0;
    PhaseDesc d;
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane(v, 0);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane(v, 1);
    d.slot_base = (int64_t)(((uint64_t)hi << 32) | lo);
    d.tile0 = __builtin_amdgcn_readlane(v, 2);
#pragma unroll
    for (int k = 0; k < kTierStar; ++k) d.T[k] = __builtin_amdgcn_readlane(v, 3 + k);
    d.sink = __builtin_amdgcn_readlane(v, 3 + kTierStar);
    return d;
}

__device__ __forceinline__ void stage_descs(int32_t nph, const PhaseDesc *descs, PhaseDesc *sd) {
    const int32_t *src = reinterpret_cast<const int32_t *>(descs);
    int32_t *dst = reinterpret_cast<int32_t *>(sd);
    const int32_t words = nph * (int32_t)(sizeof(PhaseDesc) / 4);
    for (int32_t i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
}

// Runs the wave's tiles of one LDS-tier phase: the first from the
// prefetched buffer, any further ones (phase wider than the workgroup)
// loaded into that same buffer afterwards.
template <int W, class St, bool kWeighted, class LPtr>
__device__ __forceinline__ void serial_phase(Tile<St, kWeighted> &tl, const PhaseDesc &d, int wave,
                                             int lane, const int32_t *__restrict__ tile_center,
                                             const uint32_t *__restrict__ slot_leaf,
                                             typename St::X *__restrict__ slot_x,
                                             const float *__restrict__ slot_w, LPtr L) {
    if (wave >= d.T[0]) return;
    run_tile(tl, lane, slot_x, L);
    for (int32_t t = wave + W; t < d.T[0]; t += W) {
        load_tile(tl, d, t, lane, tile_center, slot_leaf, slot_x, slot_w);
        run_tile(tl, lane, slot_x, L);
    }
}

// The phase loop of the LDS tier: phases [0, nph) whose descriptors are
// staged at sd, node loads in LDS at L (local ids), W waves.
template <int W, class St, bool kWeighted, class LPtr>
__device__ __forceinline__ void run_phases(int32_t nph, const PhaseDesc *sd, int wave, int lane,
                                           const int32_t *__restrict__ tile_center,
                                           const uint32_t *__restrict__ slot_leaf,
                                           typename St::X *__restrict__ slot_x,
                                           const float *__restrict__ slot_w, LPtr L) {
    if (nph <= 0) return;
    Tile<St, kWeighted> ta, tb;
    PhaseDesc da = desc_from_lds(sd, 0, lane), db;
    if (wave < da.T[0]) load_tile(ta, da, wave, lane, tile_center, slot_leaf, slot_x, slot_w);
    for (int32_t p = 0; p < nph; p += 2) {
        const bool has_b = p + 1 < nph;
        if (has_b) {
            db = desc_from_lds(sd, p + 1, lane);
            if (wave < db.T[0]) load_tile(tb, db, wave, lane, tile_center, slot_leaf, slot_x, slot_w);
        }
        serial_phase<W>(ta, da, wave, lane, tile_center, slot_leaf, slot_x, slot_w, L);
        lds_barrier();
        if (!has_b) break;
        if (p + 2 < nph) {
            da = desc_from_lds(sd, p + 2, lane);
            if (wave < da.T[0]) load_tile(ta, da, wave, lane, tile_center, slot_leaf, slot_x, slot_w);
        }
        serial_phase<W>(tb, db, wave, lane, tile_center, slot_leaf, slot_x, slot_w, L);
        lds_barrier();
    }
}

// The same loop without the second tile buffer: fewer registers, so more
// workgroups fit on a CU and hide each other's latency instead.
template <int W, class St, bool kWeighted, class LPtr>
__device__ __forceinline__ void run_phases_single(int32_t nph, const PhaseDesc *sd, int wave,
                                                  int lane,
                                                  const int32_t *__restrict__ tile_center,
                                                  const uint32_t *__restrict__ slot_leaf,
                                                  typename St::X *__restrict__ slot_x,
                                                  const float *__restrict__ slot_w, LPtr L) {
    Tile<St, kWeighted> tl;
    for (int32_t p = 0; p < nph; ++p) {
        const PhaseDesc d = desc_from_lds(sd, p, lane);
        for (int32_t t = wave; t < d.T[0]; t += W) {
            load_tile(tl, d, t, lane, tile_center, slot_leaf, slot_x, slot_w);
            run_tile(tl, lane, slot_x, L);
        }
        lds_barrier();
    }
}

// One middle-tier phase for this wave: its first tile's static part is
// already in tl; the loads are read now (after the previous barrier).
template <class St, bool kWeighted>
__device__ __forceinline__ void mid_phase(StationTile<St, kWeighted, kTierStar> &tl, const PhaseDesc &d,
                                          int wave, int lane, int64_t center_base,
                                          const uint32_t *__restrict__ center_next,
                                          const uint32_t *__restrict__ slot_next,
                                          typename St::X *__restrict__ slot_x,
                                          const float *__restrict__ slot_w, typename St::L *E) {
    if (wave >= d.T[0]) return;
    load_loads(tl, lane, E);
    // all loads first, on every path (see k_phase); this also completes the
    // next phase's prefetch, which the loads overtake in any case
    __builtin_amdgcn_s_waitcnt(kWaitLoads);
    run_station_tile(tl, lane, slot_x, E);
    for (int32_t t = wave + kTailWaves; t < d.T[0]; t += kTailWaves) {
        load_static(tl, d, t, lane, center_base, center_next, slot_next, slot_x, slot_w);
        load_loads(tl, lane, E);
        __builtin_amdgcn_s_waitcnt(kWaitLoads);
        run_station_tile(tl, lane, slot_x, E);
    }
}

template <class St, bool kWeighted>
__global__ void __launch_bounds__(kTailBlock)
k_mid(int32_t nph, const PhaseDesc *__restrict__ descs, int64_t center_base,
      const uint32_t *__restrict__ center_next, const uint32_t *__restrict__ slot_next,
      typename St::X *__restrict__ slot_x, const float *__restrict__ slot_w,
      typename St::L *__restrict__ E) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    PhaseDesc *sd = reinterpret_cast<PhaseDesc *>(lds_raw);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    stage_descs(nph, descs, sd);
    __syncthreads();
    if (nph <= 0) return;
    StationTile<St, kWeighted, kTierStar> ta, tb;
    PhaseDesc da = desc_from_lds(sd, 0, lane), db;
    if (wave < da.T[0])
        load_static(ta, da, wave, lane, center_base, center_next, slot_next, slot_x, slot_w);
    for (int32_t p = 0; p < nph; p += 2) {
        const bool has_b = p + 1 < nph;
        if (has_b) {
            db = desc_from_lds(sd, p + 1, lane);
            if (wave < db.T[0])
                load_static(tb, db, wave, lane, center_base, center_next, slot_next, slot_x, slot_w);
        }
        mid_phase(ta, da, wave, lane, center_base, center_next, slot_next, slot_x, slot_w, E);
        __syncthreads();
        if (!has_b) break;
        if (p + 2 < nph) {
            da = desc_from_lds(sd, p + 2, lane);
            if (wave < da.T[0])
                load_static(ta, da, wave, lane, center_base, center_next, slot_next, slot_x, slot_w);
        }
        mid_phase(tb, db, wave, lane, center_base, center_next, slot_next, slot_x, slot_w, E);
        __syncthreads();
    }
}

// The LDS tier: tail node j's load is read from its station tail_base + j,
// and written at the end to its next station tail_next[j].
template <class St, bool kWeighted>
__global__ void __launch_bounds__(kTailBlock)
k_tail(int32_t nph, const PhaseDesc *__restrict__ descs, const int32_t *__restrict__ tile_center,
       const uint32_t *__restrict__ slot_leaf, typename St::X *__restrict__ slot_x,
       const float *__restrict__ slot_w, int64_t tail_base, const uint32_t *__restrict__ tail_next,
       int32_t ntail, typename St::L *__restrict__ E) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    PhaseDesc *sd = reinterpret_cast<PhaseDesc *>(lds_raw);
    typename St::R *sL = reinterpret_cast<typename St::R *>(lds_raw + tail_desc_bytes(nph));
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    stage_descs(nph, descs, sd);
    for (int32_t i = threadIdx.x; i < ntail; i += kTailBlock) sL[i] = St::to_f64(E[tail_base + i]);
    if (threadIdx.x == 0) {
        sL[ntail] = 0.0;                    // dummy center of empty lanes
        sL[ntail + 1] = __builtin_inf();    // dummy leaf of padding rows
    }
    __syncthreads();
    run_phases<kTailWaves, St, kWeighted>(nph, sd, wave, lane, tile_center, slot_leaf, slot_x,
                                          slot_w, sL);
    __syncthreads();
    for (int32_t i = threadIdx.x; i < ntail; i += kTailBlock) E[tail_next[i]] = St::from_f64(sL[i]);
}

// ------------------------------------------------------- batched graphs --
// Many independent unweighted graphs in one persistent launch: each
// workgroup takes the next graph from a queue (graphs ordered by edge count,
// largest first), stages its loads and phase descriptors in LDS, runs
// `sweeps` sweeps of the graph's phases from LDS, and writes the loads back,
// so consecutive launches continue the same iteration.  Node ids of a graph
// are local (0..n_g-1); n_g and n_g + 1 are its dummy entries.  W waves per
// workgroup, with or without the prefetching tile buffer (the tuned launch
// shape; the result does not depend on it).
template <class St, int W, bool kPrefetch>
__global__ void __launch_bounds__(W * kWave)
k_batch(const int32_t *__restrict__ active, const int32_t *__restrict__ order,
        unsigned *__restrict__ queue,
        const int64_t *__restrict__ node_ptr, const int64_t *__restrict__ desc_ptr,
        const PhaseDesc *__restrict__ descs, const int32_t *__restrict__ tile_center,
        const uint32_t *__restrict__ slot_leaf, typename St::X *__restrict__ slot_x,
        int32_t sweeps, typename St::L *__restrict__ Lstate) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ int32_t s_graph;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    const unsigned G = (unsigned)*active;   // graphs still iterating, order[0..G)
    for (;;) {
        if (threadIdx.x == 0) {
            const unsigned k = atomicAdd(queue, 1u);
            s_graph = k < G ? order[k] : -1;
        }
        __syncthreads();
        const int32_t g = s_graph;
        if (g < 0) break;
        const int64_t n0 = node_ptr[g];
        const int32_t n = (int32_t)(node_ptr[g + 1] - n0);
        const int32_t nph = (int32_t)(desc_ptr[g + 1] - desc_ptr[g]);
        PhaseDesc *sd = reinterpret_cast<PhaseDesc *>(lds_raw);
        typename St::R *sL = reinterpret_cast<typename St::R *>(lds_raw + tail_desc_bytes(nph));
        stage_descs(nph, descs + desc_ptr[g], sd);
        for (int32_t u = threadIdx.x; u < n; u += W * kWave) sL[u] = St::to_f64(Lstate[n0 + u]);
        if (threadIdx.x == 0) {
            sL[n] = 0.0;
            sL[n + 1] = __builtin_inf();
        }
        __syncthreads();
        for (int32_t t = 0; t < sweeps; ++t) {
            if (kPrefetch)
                run_phases<W, St, false>(nph, sd, wave, lane, tile_center, slot_leaf, slot_x,
                                         nullptr, sL);
            else
                run_phases_single<W, St, false>(nph, sd, wave, lane, tile_center, slot_leaf,
                                                slot_x, nullptr, sL);
        }
        __syncthreads();
        for (int32_t u = threadIdx.x; u < n; u += W * kWave) Lstate[n0 + u] = St::from_f64(sL[u]);
        __syncthreads();   // LDS reuse by the next graph
    }
}

// ------------------------------------------- batched solve in one launch --
// Each workgroup takes the next graph from the queue and solves it to the
// tolerance on its own: sweeps from LDS (as k_batch), then, every few
// sweeps, the check of Section III-B inside the workgroup (wg_check.h): the
// loads' maximum D, the dual bound; when D does not already certify the
// densest set found so far, Algorithm 1's extraction (a stable radix sort
// of the loads, each node's count of neighbours at higher positions, the
// densest removal prefix); the graph stops once (D - rho_best) / rho_best
// <= tol or at max_sweeps.  FP32K screens with the kept loads and confirms
// a passing gap with D of the loads recomputed from the stored fractions.  Between
// checks the cadence follows the decay of the gap (wg_next_check).  No
// kernel boundary or host round trip falls inside a solve, so a graph stops
// at its own check and not at a launch boundary.
template <class St, int W, bool kPrefetch>
__global__ void __launch_bounds__(W * kWave) k_batch_solve(BatchSolveArgs a) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ int32_t s_graph;
    __shared__ WgCheckLds<W> ls;
    using X = typename St::X;
    using L = typename St::L;
    X *slot_x = (X *)a.slot_x;
    L *Lstate = (L *)a.Lstate;
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(tid / kWave);
    const unsigned G = (unsigned)*a.active;
    for (;;) {
        if (tid == 0) {
            const unsigned k = atomicAdd(a.queue, 1u);
            s_graph = k < G ? a.order[k] : -1;
        }
        __syncthreads();
        const int32_t g = s_graph;
        if (g < 0) break;
        const int64_t n0 = a.node_ptr[g];
        const int32_t n = (int32_t)(a.node_ptr[g + 1] - n0);
        const int32_t nph = (int32_t)(a.desc_ptr[g + 1] - a.desc_ptr[g]);
        PhaseDesc *sd = reinterpret_cast<PhaseDesc *>(lds_raw);
        typename St::R *sL = reinterpret_cast<typename St::R *>(lds_raw + tail_desc_bytes(nph));
        stage_descs(nph, a.descs + a.desc_ptr[g], sd);
        for (int32_t u = tid; u < n; u += W * kWave) sL[u] = St::to_f64(Lstate[n0 + u]);
        if (tid == 0) {
            sL[n] = 0.0;
            sL[n + 1] = __builtin_inf();
        }
        __syncthreads();
        uint64_t *k0 = a.k0 + n0, *k1 = a.k1 + n0;
        uint32_t *i0 = a.i0 + n0, *i1 = a.i1 + n0;
        int32_t *pos = a.pos + n0, *hist = a.hist + n0;
        int32_t sweeps = 0, k = a.check_every, t0 = -1, t1 = -1, set_at = 0;
        double g0 = 0.0, g1 = 0.0, gap = 1.0e300, D = 0.0;
        int64_t bnum = 0, bden = 0;
        bool have = false;
        for (;;) {
            const int32_t kk = k < a.max_sweeps - sweeps ? k : a.max_sweeps - sweeps;
            for (int32_t t = 0; t < kk; ++t) {
                if (kPrefetch)
                    run_phases<W, St, false>(nph, sd, wave, lane, a.tile_center, a.slot_leaf,
                                             slot_x, nullptr, sL);
                else
                    run_phases_single<W, St, false>(nph, sd, wave, lane, a.tile_center,
                                                    a.slot_leaf, slot_x, nullptr, sL);
            }
            sweeps += kk;
            // every wave's fraction stores are complete and visible before the
            // fractions are read back
            __syncthreads();
            // FP64 loads as sort keys, and their maximum D (for FP32K the
            // loads as kept: they screen; a passing gap is confirmed below)
            double vmax = -1.0e308;
            for (int32_t u = tid; u < n; u += W * kWave) {
                const double v = sL[u];
                k0[u] = wg_sortable(v);
                i0[u] = (uint32_t)u;
                vmax = v > vmax ? v : vmax;
            }
            D = wg_max<W>(vmax, ls);
            bool certified = false;
            if (have) {
                gap = batch_rel_gap(D, bnum, bden);
                certified = gap <= a.tol;
            }
            if (!certified) {
                const bool in1 = wg_radix_sort<W>(k0, i0, k1, i1, n, ls);
                const uint32_t *ids = in1 ? i1 : i0;
                for (int32_t i = tid; i < n; i += W * kWave) pos[ids[i]] = i;
                __syncthreads();
                for (int32_t u = tid; u < n; u += W * kWave) {
                    const int32_t p = pos[u];
                    int32_t c = 0;
                    for (int64_t j = a.row_ptr[n0 + u]; j < a.row_ptr[n0 + u + 1]; ++j)
                        c += pos[a.adj[j] - n0] > p ? 1 : 0;
                    hist[p] = c;
                }
                __syncthreads();
                int64_t bi, bw;
                wg_best_prefix<W>(hist, n, ls, &bi, &bw);
                const int64_t en = bw, ed = (int64_t)n - bi;
                if (!have || (__int128)en * bden >= (__int128)bnum * ed) {
                    have = true;
                    bnum = en;
                    bden = ed;
                    set_at = sweeps;
                    for (int32_t u = tid; u < n; u += W * kWave)
                        a.in_set[n0 + u] = pos[u] >= bi ? 1 : 0;
                }
                gap = batch_rel_gap(D, bnum, bden);
            }
            if (St::kRecompute && gap <= a.tol) {
                // only the loads of the stored fractions make a feasible dual
                // point: D from those (FP64 sums along each node's incidence,
                // 8 lanes a node, fixed order), and the carried loads restart
                // from them, so a failed confirmation leaves no drift behind
                double emax = -1.0e308;
                const int sub = tid & (kRowLanes - 1);
                for (int32_t u0 = tid / kRowLanes; u0 < n; u0 += W * kWave / kRowLanes) {
                    const int64_t b = a.row_ptr[n0 + u0], e = a.row_ptr[n0 + u0 + 1];
                    double v = 0.0;
                    for (int64_t j = b + sub; j < e; j += kRowLanes) {
                        const uint32_t ent = a.inc_slot[j];
                        const double x = (double)slot_x[ent >> 1];
                        v = v + ((ent & 1u) ? 1.0 - x : x);
                    }
                    for (int d = kRowLanes / 2; d > 0; d >>= 1) v = v + __shfl_down(v, d, kRowLanes);
                    if (sub == 0) {
                        sL[u0] = v;
                        emax = v > emax ? v : emax;
                    }
                }
                D = wg_max<W>(emax, ls);
                gap = batch_rel_gap(D, bnum, bden);
            }
            if (gap <= a.tol || sweeps >= a.max_sweeps) break;
            t0 = t1;
            g0 = g1;
            t1 = sweeps;
            g1 = gap;
            k = wg_next_check(t0, g0, t1, g1, a.tol, a.check_every);
        }
        __syncthreads();
        for (int32_t u = tid; u < n; u += W * kWave) Lstate[n0 + u] = St::from_f64(sL[u]);
        if (tid == 0) {
            a.num[g] = bnum;
            a.den[g] = bden;
            a.D[g] = D;
            a.sweeps_used[g] = sweeps;
            a.set_sweeps[g] = set_at;
            if (gap > a.tol) atomicAdd(a.queue + 1, 1u);
        }
        __syncthreads();   // LDS reuse by the next graph
    }
}

// Retires converged graphs: keeps, in order, the graphs of `all` whose
// relative gap (D_g - rho_g) / rho_g with rho_g = num_g / den_g exceeds tol
// (a graph without edges has D_g = rho_g = 0 and is converged); writes the
// kept list, its length and its edge count.  One workgroup.
constexpr int kRetireBlock = 1024;
__global__ void __launch_bounds__(kRetireBlock)
k_retire(int32_t G, const int32_t *all, const int64_t *edge_ptr, const int64_t *num,
         const int64_t *den, const double *D, double tol, int32_t *order, int32_t *active,
         int64_t *active_edges) {
    __shared__ int32_t s_cnt[kRetireBlock];
    __shared__ int64_t s_edges[kRetireBlock];
    __shared__ int32_t s_base;
    __shared__ int64_t s_etot;
    if (threadIdx.x == 0) {
        s_base = 0;
        s_etot = 0;
    }
    __syncthreads();
    for (int32_t i0 = 0; i0 < G; i0 += kRetireBlock) {
        const int32_t i = i0 + (int32_t)threadIdx.x;
        int32_t keep = 0, g = -1;
        if (i < G) {
            g = all[i];
            const double rho = (double)num[g] / (double)den[g];
            const double gap = rho > 0.0 ? (D[g] - rho) / rho : (D[g] > 0.0 ? 1.0e300 : 0.0);
            keep = gap > tol ? 1 : 0;
        }
        s_cnt[threadIdx.x] = keep;
        s_edges[threadIdx.x] = keep ? edge_ptr[g + 1] - edge_ptr[g] : 0;
        __syncthreads();
        // inclusive scan of the flags (Hillis-Steele in LDS) and sum of edges
        for (int d = 1; d < kRetireBlock; d <<= 1) {
            const int32_t a = threadIdx.x >= (unsigned)d ? s_cnt[threadIdx.x - d] : 0;
            const int64_t b = threadIdx.x >= (unsigned)d ? s_edges[threadIdx.x - d] : 0;
            __syncthreads();
            s_cnt[threadIdx.x] += a;
            s_edges[threadIdx.x] += b;
            __syncthreads();
        }
        if (keep) order[s_base + s_cnt[threadIdx.x] - 1] = g;
        __syncthreads();
        if (threadIdx.x == 0) {
            s_base += s_cnt[kRetireBlock - 1];
            s_etot += s_edges[kRetireBlock - 1];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *active = s_base;
        *active_edges = s_etot;
    }
}

// the full list again (a reset)
__global__ void k_activate_all(int32_t G, const int32_t *all, const int64_t *edge_ptr,
                               int32_t *order, int32_t *active, int64_t *active_edges) {
    for (int32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < G; i += gridDim.x * blockDim.x)
        order[i] = all[i];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        *active = G;
        *active_edges = edge_ptr[G];
    }
}

// Initial loads of a batch: deg(u) / 2 (a sum of halves, exact).
__global__ void k_batch_degrees(int64_t M, const int32_t *gsrc, const int32_t *gdst,
                                int32_t *deg) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < M;
         e += (int64_t)gridDim.x * blockDim.x) {
        atomicAdd(&deg[gsrc[e]], 1);
        atomicAdd(&deg[gdst[e]], 1);
    }
}

template <class St>
__global__ void k_batch_init_loads(int64_t N, const int32_t *deg, typename St::L *Lstate) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < N;
         u += (int64_t)gridDim.x * blockDim.x)
        Lstate[u] = St::from_f64((double)deg[u] * 0.5);
}

template <class St>
__global__ void k_batch_loads_f64(int64_t N, const typename St::L *Lstate, double *L64) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < N;
         u += (int64_t)gridDim.x * blockDim.x)
        L64[u] = St::to_f64(Lstate[u]);
}

__global__ void k_zero_u32(unsigned *p) { *p = 0u; }
__global__ void k_zero_u32x2(unsigned *p) {
    p[0] = 0u;
    p[1] = 0u;
}

// ------------------------------------------------------------ statistics --
constexpr int kRedBlock = 256;

// FP64 loads recomputed from the fractions (f_e(src) = x, f_e(dst) = w - x):
// a group of kRowLanes lanes per node of degree below kBigRow, lanes striding
// over the row, fixed-order reduction; longer rows: k_recompute_big.
template <class St, bool kWeighted>
__device__ __forceinline__ double recompute_term(uint32_t ent, const int64_t *edge_slot,
                                                 const typename St::X *slot_x, const float *w) {
    const int64_t e = ent >> 1;
    const double x = (double)slot_x[edge_slot[e]];
    const double we = kWeighted ? (double)w[e] : 1.0;
    return (ent & 1) ? we - x : x;
}

template <class St, bool kWeighted>
__global__ void __launch_bounds__(256) k_recompute(int32_t n, const int64_t *row_ptr,
                                                   const uint32_t *inc, const int64_t *edge_slot,
                                                   const typename St::X *slot_x, const float *w,
                                                   double *L64) {
    const int sub = threadIdx.x & (kRowLanes - 1);
    const int64_t groups = (int64_t)gridDim.x * (blockDim.x / kRowLanes);
    for (int64_t u = (int64_t)blockIdx.x * (blockDim.x / kRowLanes) + threadIdx.x / kRowLanes;
         u < n; u += groups) {
        const int64_t b = row_ptr[u], e = row_ptr[u + 1];
        if (e - b >= kBigRow) continue;
        double acc = 0.0;
        for (int64_t j = b + sub; j < e; j += kRowLanes)
            acc = acc + recompute_term<St, kWeighted>(inc[j], edge_slot, slot_x, w);
        for (int d = kRowLanes / 2; d > 0; d >>= 1) acc = acc + __shfl_down(acc, d, kRowLanes);
        if (sub == 0) L64[u] = acc;
    }
}

// Batches (unit weights): the same per-node sums for the nodes of the
// graphs still iterating (flag[node_graph[u]] set, see k_mark_active), 8
// lanes per node for every row (a batch's graphs have no long rows to speak
// of); written to L64 and, rounded to the state's load type, as the carried
// loads.  Retired graphs keep both from their last pass: their
// fractions no longer change.
template <class St>
__global__ void __launch_bounds__(256)
k_batch_recompute(int64_t N, const int32_t *node_graph, const uint8_t *flag,
                  const int64_t *row_ptr, const uint32_t *inc, const int64_t *edge_slot,
                  const typename St::X *slot_x, double *L64, typename St::L *Lstate) {
    const int sub = threadIdx.x & (kRowLanes - 1);
    const int64_t groups = (int64_t)gridDim.x * (blockDim.x / kRowLanes);
    for (int64_t u = (int64_t)blockIdx.x * (blockDim.x / kRowLanes) + threadIdx.x / kRowLanes;
         u < N; u += groups) {
        if (!flag[node_graph[u]]) continue;   // the whole 8-lane group skips together
        const int64_t b = row_ptr[u], e = row_ptr[u + 1];
        double acc = 0.0;
        for (int64_t j = b + sub; j < e; j += kRowLanes)
            acc = acc + recompute_term<St, false>(inc[j], edge_slot, slot_x, nullptr);
        for (int d = kRowLanes / 2; d > 0; d >>= 1) acc = acc + __shfl_down(acc, d, kRowLanes);
        if (sub == 0) {
            L64[u] = acc;
            Lstate[u] = St::from_f64(acc);
        }
    }
}

// Each incidence entry's slot: (slot of its edge) << 1 | side, so the sums of
// the fractions along a row take one gather per entry.
__global__ void k_inc_slots(int64_t entries, const uint32_t *inc, const int64_t *edge_slot,
                            uint32_t *inc_slot) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < entries;
         j += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t ent = inc[j];
        inc_slot[j] = ((uint32_t)edge_slot[ent >> 1] << 1) | (ent & 1u);
    }
}

// flag[g] = 1 for the graphs order[0..*active), 0 for the others.  One
// workgroup.
constexpr int kMarkBlock = 1024;
__global__ void __launch_bounds__(kMarkBlock)
k_mark_active(int32_t G, const int32_t *active, const int32_t *order, uint8_t *flag) {
    for (int32_t g = threadIdx.x; g < G; g += kMarkBlock) flag[g] = 0;
    __syncthreads();
    const int32_t A = *active;
    for (int32_t i = threadIdx.x; i < A; i += kMarkBlock) flag[order[i]] = 1;
}

constexpr int kBigRowBlock = 256;
template <class St, bool kWeighted>
__global__ void __launch_bounds__(kBigRowBlock) k_recompute_big(
    const int32_t *big, const int64_t *row_ptr, const uint32_t *inc, const int64_t *edge_slot,
    const typename St::X *slot_x, const float *w, double *L64) {
    __shared__ double part[kBigRowBlock / kWave];
    const int32_t u = big[blockIdx.x];
    double acc = 0.0;
    for (int64_t j = row_ptr[u] + threadIdx.x; j < row_ptr[u + 1]; j += kBigRowBlock)
        acc = acc + recompute_term<St, kWeighted>(inc[j], edge_slot, slot_x, w);
    for (int d = kWave / 2; d > 0; d >>= 1) acc = acc + __shfl_down(acc, d, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
        for (int k = 0; k < kBigRowBlock / kWave; ++k) t = t + part[k];
        L64[u] = t;
    }
}

// the current load of every node, read at its first station (between sweeps)
template <class St>
__global__ void k_loads_to_f64(int32_t n, const uint32_t *home, const typename St::L *E,
                               double *L64) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x)
        L64[u] = St::to_f64(E[home[u]]);
}

// The inverse: node u's carried load set from an FP64 value.
template <class St>
__global__ void k_loads_from_f64(int32_t n, const uint32_t *home, const double *L64,
                                 typename St::L *E) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x)
        E[home[u]] = St::from_f64(L64[u]);
}

__device__ inline void red3(double &mx, double &s, double &s2, double *lds) {
    // block reduction of (max, sum, sum of squares); fixed order
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    for (int d = kWave / 2; d > 0; d >>= 1) {
        double a = __shfl_down(mx, d, kWave), b = __shfl_down(s, d, kWave),
               c = __shfl_down(s2, d, kWave);
        mx = a > mx ? a : mx;
        s = s + b;
        s2 = s2 + c;
    }
    if (lane == 0) {
        lds[wave * 3 + 0] = mx;
        lds[wave * 3 + 1] = s;
        lds[wave * 3 + 2] = s2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < (int)(blockDim.x / kWave); ++k) {
            mx = lds[k * 3] > mx ? lds[k * 3] : mx;
            s = s + lds[k * 3 + 1];
            s2 = s2 + lds[k * 3 + 2];
        }
    }
}

__global__ void __launch_bounds__(kRedBlock) k_stats_partial(int64_t n, const double *L,
                                                             double *partial) {
    __shared__ double lds[3 * (kRedBlock / kWave)];
    double mx = -1.0e308, s = 0.0, s2 = 0.0;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x) {
        double v = L[u];
        mx = v > mx ? v : mx;
        s = s + v;
        s2 = s2 + v * v;
    }
    red3(mx, s, s2, lds);
    if (threadIdx.x == 0) {
        partial[blockIdx.x * 3 + 0] = mx;
        partial[blockIdx.x * 3 + 1] = s;
        partial[blockIdx.x * 3 + 2] = s2;
    }
}

__global__ void __launch_bounds__(kRedBlock) k_stats_final(int32_t nb, const double *partial,
                                                           double *out) {
    __shared__ double lds[3 * (kRedBlock / kWave)];
    double mx = -1.0e308, s = 0.0, s2 = 0.0;
    for (int32_t b = threadIdx.x; b < nb; b += blockDim.x) {
        mx = partial[b * 3] > mx ? partial[b * 3] : mx;
        s = s + partial[b * 3 + 1];
        s2 = s2 + partial[b * 3 + 2];
    }
    red3(mx, s, s2, lds);
    if (threadIdx.x == 0) {
        out[0] = mx;
        out[1] = s;
        out[2] = s2;
    }
}

template <class St>
__global__ void k_read_x(int64_t m, const int64_t *edge_slot, const typename St::X *slot_x,
                         double *x) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x)
        x[e] = (double)slot_x[edge_slot[e]];
}

}  // namespace

// ------------------------------------------------------------ launchers --
template <class St, bool kW>
static void sweep_launchers(SweepLaunch &fn) {
    fn.init_slots = [](int64_t nslots, const int64_t *slot_edge, const float *w, void *slot_x,
                       float *slot_w, hipStream_t s) {
        hipLaunchKernelGGL((k_init_slots<St, kW>), dim3(grid_for(nslots, 256)), dim3(256), 0, s,
                           nslots, slot_edge, w, (typename St::X *)slot_x, slot_w);
    };
    fn.init_loads = [](int32_t n, const int64_t *row_ptr, const uint32_t *inc, const float *w,
                       const uint32_t *home, const int32_t *big, int32_t nbig, int64_t entries,
                       int64_t center_base, void *E, hipStream_t s) {
        hipLaunchKernelGGL((k_fill_entries<St>), dim3(grid_for(entries, 256)), dim3(256), 0, s,
                           entries, center_base, (typename St::L *)E);
        hipLaunchKernelGGL((k_init_loads<St, kW>), dim3(grid_for((int64_t)n, 256)), dim3(256), 0, s,
                           n, row_ptr, inc, w, home, (typename St::L *)E);
        if (kW && nbig > 0)
            hipLaunchKernelGGL((k_init_loads_big<St>), dim3((unsigned)nbig), dim3(kWave), 0, s, big,
                               row_ptr, inc, w, home, (typename St::L *)E);
    };
    fn.phase = [](const PhaseDescWide &d, int64_t center_base, const uint32_t *center_next,
                  const uint32_t *slot_next, void *slot_x, const float *slot_w, void *E,
                  const uint32_t *slot_src, const uint32_t *center_src, hipStream_t s) {
        const int32_t tiles = d.T[0];
        int32_t spread = 0;
        while (spread < kMaxSpreadLog2 && ((int64_t)tiles << (spread + 1)) <= kSpreadWaves)
            ++spread;
        const unsigned blocks = (unsigned)((int64_t)tiles << spread);
        const bool pull = slot_src != nullptr;
        if (desc_depth(d) <= kTierStar) {
            const PhaseDesc n = narrow_desc<kTierStar>(d);
            if (pull)
                hipLaunchKernelGGL((k_phase<St, kW, kTierStar, true>), dim3(blocks),
                                   dim3(kPhaseBlock), 0, s, n.slot_base, n.tile0, n.T[0],
                                   n.T[kTierStar - 1], spread, center_base, (typename St::L *)E,
                                   slot_next, (typename St::X *)slot_x, center_next, n, slot_w,
                                   slot_src, center_src);
            else
                hipLaunchKernelGGL((k_phase<St, kW, kTierStar, false>), dim3(blocks),
                                   dim3(kPhaseBlock), 0, s, n.slot_base, n.tile0, n.T[0],
                                   n.T[kTierStar - 1], spread, center_base, (typename St::L *)E,
                                   slot_next, (typename St::X *)slot_x, center_next, n, slot_w,
                                   nullptr, nullptr);
        } else {
            if (pull)
                hipLaunchKernelGGL((k_phase<St, kW, kMaxStar, true>), dim3(blocks),
                                   dim3(kPhaseBlock), 0, s, d.slot_base, d.tile0, d.T[0],
                                   d.T[kMaxStar - 1], spread, center_base, (typename St::L *)E,
                                   slot_next, (typename St::X *)slot_x, center_next, d, slot_w,
                                   slot_src, center_src);
            else
                hipLaunchKernelGGL((k_phase<St, kW, kMaxStar, false>), dim3(blocks),
                                   dim3(kPhaseBlock), 0, s, d.slot_base, d.tile0, d.T[0],
                                   d.T[kMaxStar - 1], spread, center_base, (typename St::L *)E,
                                   slot_next, (typename St::X *)slot_x, center_next, d, slot_w,
                                   nullptr, nullptr);
        }
    };
    fn.phase_node = [](const PhaseDescWide &d, const int32_t *tile_center,
                       const uint32_t *slot_leaf, void *slot_x, const float *slot_w, void *E,
                       hipStream_t s) {
        const int32_t tiles = d.T[0];
        int32_t spread = 0;
        while (spread < kMaxSpreadLog2 && ((int64_t)tiles << (spread + 1)) <= kSpreadWaves)
            ++spread;
        const unsigned blocks = (unsigned)((int64_t)tiles << spread);
        if (desc_depth(d) <= kTierStar)
            hipLaunchKernelGGL((k_phase_node<St, kW, kTierStar>), dim3(blocks), dim3(kPhaseBlock),
                               0, s, narrow_desc<kTierStar>(d), spread, tile_center, slot_leaf,
                               (typename St::X *)slot_x, slot_w, (typename St::L *)E);
        else
            hipLaunchKernelGGL((k_phase_node<St, kW, kMaxStar>), dim3(blocks), dim3(kPhaseBlock), 0,
                               s, d, spread, tile_center, slot_leaf, (typename St::X *)slot_x,
                               slot_w, (typename St::L *)E);
    };
    fn.fill_nodes = [](int32_t n, void *E, hipStream_t s) {
        hipLaunchKernelGGL((k_fill_nodes<St>), dim3(grid_for((int64_t)n + 2, 256)), dim3(256), 0, s,
                           n, (typename St::L *)E);
    };
    fn.tail = [](int32_t nph, const PhaseDesc *descs, const int32_t *tile_center,
                 const uint32_t *slot_leaf, void *slot_x, const float *slot_w, int64_t tail_base,
                 const uint32_t *tail_next, int32_t ntail, void *E, hipStream_t s) {
        size_t lds = tail_desc_bytes(nph) + (size_t)(ntail + 2) * sizeof(typename St::R);
        hipLaunchKernelGGL((k_tail<St, kW>), dim3(1), dim3(kTailBlock), lds, s, nph, descs,
                           tile_center, slot_leaf, (typename St::X *)slot_x, slot_w, tail_base,
                           tail_next, ntail, (typename St::L *)E);
    };
    fn.mid = [](int32_t nph, const PhaseDesc *descs, int64_t center_base,
                const uint32_t *center_next, const uint32_t *slot_next, void *slot_x,
                const float *slot_w, void *E, hipStream_t s) {
        size_t lds = tail_desc_bytes(nph);
        hipLaunchKernelGGL((k_mid<St, kW>), dim3(1), dim3(kTailBlock), lds, s, nph, descs,
                           center_base, center_next, slot_next, (typename St::X *)slot_x, slot_w,
                           (typename St::L *)E);
    };
    fn.set_tail_lds = [](size_t bytes) {
        LOWD_HIP(hipFuncSetAttribute((const void *)k_tail<St, kW>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    };
    fn.set_mid_lds = [](size_t bytes) {
        LOWD_HIP(hipFuncSetAttribute((const void *)k_mid<St, kW>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    };
    fn.loads_f64 = [](int32_t n, const int64_t *row_ptr, const uint32_t *inc,
                      const int64_t *edge_slot, const void *slot_x, const float *w,
                      const uint32_t *home, const int32_t *big, int32_t nbig, const void *E,
                      double *L64, hipStream_t s) {
        if (St::kRecompute) {
            hipLaunchKernelGGL((k_recompute<St, kW>), dim3(grid_for((int64_t)n * kRowLanes, 256)),
                               dim3(256), 0, s, n, row_ptr, inc, edge_slot,
                               (const typename St::X *)slot_x, w, L64);
            if (nbig > 0)
                hipLaunchKernelGGL((k_recompute_big<St, kW>), dim3((unsigned)nbig),
                                   dim3(kBigRowBlock), 0, s, big, row_ptr, inc, edge_slot,
                                   (const typename St::X *)slot_x, w, L64);
        } else
            hipLaunchKernelGGL((k_loads_to_f64<St>), dim3(grid_for(n, 256)), dim3(256), 0, s, n,
                               home, (const typename St::L *)E, L64);
    };
    fn.write_loads = [](int32_t n, const uint32_t *home, const double *L64, void *E,
                        hipStream_t s) {
        hipLaunchKernelGGL((k_loads_from_f64<St>), dim3(grid_for(n, 256)), dim3(256), 0, s, n,
                           home, L64, (typename St::L *)E);
    };
    fn.read_x = [](int64_t m, const int64_t *edge_slot, const void *slot_x, double *x,
                   hipStream_t s) {
        hipLaunchKernelGGL((k_read_x<St>), dim3(grid_for(m, 256)), dim3(256), 0, s, m, edge_slot,
                           (const typename St::X *)slot_x, x);
    };
    fn.read_loads = [](int32_t n, const uint32_t *home, const void *E, double *out,
                       hipStream_t s) {
        hipLaunchKernelGGL((k_loads_to_f64<St>), dim3(grid_for(n, 256)), dim3(256), 0, s, n, home,
                           (const typename St::L *)E, out);
    };
    fn.batch = [](int32_t shape, const int32_t *active, const int32_t *order, unsigned *queue,
                  const int64_t *node_ptr, const int64_t *desc_ptr, const PhaseDesc *descs,
                  const int32_t *tile_center, const uint32_t *slot_leaf, void *slot_x,
                  int32_t sweeps, void *Lstate, size_t lds, int32_t blocks, hipStream_t s) {
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, queue);
#define LOWD_BATCH_CASE(W, PF)                                                                 \
    case W * 2 + PF:                                                                           \
        hipLaunchKernelGGL((k_batch<St, W, PF>), dim3((unsigned)blocks), dim3(W * kWave), lds,  \
                           s, active, order, queue, node_ptr, desc_ptr, descs, tile_center,    \
                           slot_leaf, (typename St::X *)slot_x, sweeps,                        \
                           (typename St::L *)Lstate);                                          \
        break;
        switch (shape) {
            LOWD_BATCH_CASE(4, 0)
            LOWD_BATCH_CASE(4, 1)
            LOWD_BATCH_CASE(8, 0)
            LOWD_BATCH_CASE(8, 1)
            LOWD_BATCH_CASE(16, 0)
            default: fail(LOWD_E_ARG, "unsupported batch workgroup shape");
        }
#undef LOWD_BATCH_CASE
    };
    fn.set_batch_lds = [](int32_t shape, size_t bytes) {
        const void *k = shape == 8 ? (const void *)k_batch<St, 4, false>
                        : shape == 9 ? (const void *)k_batch<St, 4, true>
                        : shape == 16 ? (const void *)k_batch<St, 8, false>
                        : shape == 17 ? (const void *)k_batch<St, 8, true>
                        : shape == 32 ? (const void *)k_batch<St, 16, false>
                                      : nullptr;
        if (!k) fail(LOWD_E_ARG, "unsupported batch workgroup shape");
        LOWD_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    };
    fn.batch_solve = [](int32_t shape, const BatchSolveArgs &a, size_t lds, int32_t blocks,
                        hipStream_t s) {
        hipLaunchKernelGGL(k_zero_u32x2, dim3(1), dim3(1), 0, s, a.queue);
#define LOWD_SOLVE_CASE(W, PF)                                                                 \
    case W * 2 + PF:                                                                           \
        hipLaunchKernelGGL((k_batch_solve<St, W, PF>), dim3((unsigned)blocks), dim3(W * kWave),  \
                           lds, s, a);                                                         \
        break;
        switch (shape) {   // the shapes whose sweeps and checks fit 256 registers
            LOWD_SOLVE_CASE(4, 0)
            LOWD_SOLVE_CASE(4, 1)
            LOWD_SOLVE_CASE(8, 0)
            default: fail(LOWD_E_ARG, "unsupported batch workgroup shape for the solve");
        }
#undef LOWD_SOLVE_CASE
    };
    fn.set_batch_solve_lds = [](int32_t shape, size_t bytes) {
        const void *k = shape == 8 ? (const void *)k_batch_solve<St, 4, false>
                        : shape == 9 ? (const void *)k_batch_solve<St, 4, true>
                        : shape == 16 ? (const void *)k_batch_solve<St, 8, false>
                                      : nullptr;
        if (!k) fail(LOWD_E_ARG, "unsupported batch workgroup shape for the solve");
        LOWD_HIP(hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    };
    fn.batch_init_loads = [](int64_t N, const int32_t *deg, void *Lstate, hipStream_t s) {
        hipLaunchKernelGGL((k_batch_init_loads<St>), dim3(grid_for(N, 256)), dim3(256), 0, s, N,
                           deg, (typename St::L *)Lstate);
    };
    fn.batch_loads_f64 = [](int64_t N, const void *Lstate, double *L64, hipStream_t s) {
        hipLaunchKernelGGL((k_batch_loads_f64<St>), dim3(grid_for(N, 256)), dim3(256), 0, s, N,
                           (const typename St::L *)Lstate, L64);
    };
    fn.batch_recompute = [](int32_t G, int64_t N, const int32_t *active, const int32_t *order,
                            const int32_t *node_graph, uint8_t *flag, const int64_t *row_ptr,
                            const uint32_t *inc, const int64_t *edge_slot, const void *slot_x,
                            double *L64, void *Lstate, hipStream_t s) {
        hipLaunchKernelGGL(k_mark_active, dim3(1), dim3(kMarkBlock), 0, s, G, active, order, flag);
        hipLaunchKernelGGL((k_batch_recompute<St>), dim3(grid_for(N * kRowLanes, 256)), dim3(256),
                           0, s, N, node_graph, flag, row_ptr, inc, edge_slot,
                           (const typename St::X *)slot_x, L64, (typename St::L *)Lstate);
    };
    fn.x_bytes = sizeof(typename St::X);
    // a load takes as many bytes at rest as in LDS: l_bytes sizes both
    static_assert(sizeof(typename St::L) == sizeof(typename St::R), "load sizes");
    fn.l_bytes = sizeof(typename St::L);
}

void get_sweep_launchers(int32_t state, bool weighted, SweepLaunch &fn) {
    if (state == 0) {
        if (weighted) sweep_launchers<StateF64, true>(fn);
        else sweep_launchers<StateF64, false>(fn);
    } else {
        if (weighted) sweep_launchers<StateF32K, true>(fn);
        else sweep_launchers<StateF32K, false>(fn);
    }
}

void launch_inc_slots(int64_t entries, const uint32_t *inc, const int64_t *edge_slot,
                      uint32_t *inc_slot, hipStream_t s) {
    if (entries > 0)
        hipLaunchKernelGGL(k_inc_slots, dim3(grid_for(entries, 256)), dim3(256), 0, s, entries,
                           inc, edge_slot, inc_slot);
}

void launch_retire(int32_t G, const int32_t *all, const int64_t *edge_ptr, const int64_t *num,
                   const int64_t *den, const double *D, double tol, int32_t *order,
                   int32_t *active, int64_t *active_edges, hipStream_t s) {
    hipLaunchKernelGGL(k_retire, dim3(1), dim3(kRetireBlock), 0, s, G, all, edge_ptr, num, den, D,
                       tol, order, active, active_edges);
}

void launch_activate_all(int32_t G, const int32_t *all, const int64_t *edge_ptr, int32_t *order,
                         int32_t *active, int64_t *active_edges, hipStream_t s) {
    hipLaunchKernelGGL(k_activate_all, dim3(grid_for(G, 256)), dim3(256), 0, s, G, all, edge_ptr,
                       order, active, active_edges);
}

void launch_batch_degrees(int64_t N, int64_t M, const int32_t *gsrc, const int32_t *gdst,
                          int32_t *deg, hipStream_t s) {
    LOWD_HIP(hipMemsetAsync(deg, 0, (size_t)(N > 0 ? N : 1) * sizeof(int32_t), s));
    if (M > 0)
        hipLaunchKernelGGL(k_batch_degrees, dim3(grid_for(M, 256)), dim3(256), 0, s, M, gsrc, gdst,
                           deg);
}

void launch_stats(int64_t n, const double *L64, double *partial, int32_t nb, double *out,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_stats_partial, dim3((unsigned)nb), dim3(kRedBlock), 0, s, n, L64, partial);
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(kRedBlock), 0, s, nb, partial, out);
}

}  // namespace lowd
