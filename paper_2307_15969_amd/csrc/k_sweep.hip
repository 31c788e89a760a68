// k_sweep.hip -- initialisation, the LOWD edge sweep and its convergence
// statistics.
//
// The sweep follows the phase schedule (schedule.cpp): one kernel per phase
// for the wide phases; the narrow last phases run inside one workgroup that
// keeps their nodes' loads in LDS.  Inside a phase every lane owns one star:
// it keeps the center's load in a register, and walks the star's leaves in
// order, applying Algorithm 1's locally optimal step to each edge.  The
// stars of a phase share no node, so no atomics are needed and the result is
// that of the sequential edge loop in schedule order.
#include "lowd_internal.h"
#include "sweep_state.h"

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

// l_u = sum of w_e / 2 over the edges at u, in ascending edge index; entry
// n (the dummy center of lanes without a star) is zero and entry n+1 (the
// dummy leaf of padding rows) is +infinity
template <class St, bool kWeighted>
__global__ void k_init_loads(int32_t n, const int64_t *row_ptr, const uint32_t *inc,
                             const float *w, typename St::L *L) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u <= n + 1;
         u += (int64_t)gridDim.x * blockDim.x) {
        if (u == n + 1) {
            L[u] = St::infinite();
            continue;
        }
        double acc = 0.0;
        if (u < n) {
            if (kWeighted) {
                for (int64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j)
                    acc = acc + (double)w[inc[j] >> 1] / 2.0;
            } else {
                // a sum of halves is exact in any order: deg / 2
                acc = (double)(row_ptr[u + 1] - row_ptr[u]) * 0.5;
            }
        }
        L[u] = St::from_f64(acc);
    }
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
    uint32_t enc[kMaxStar];
    typename St::X x[kMaxStar];
    float w[kMaxStar];
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
    for (int k = 0; k < kMaxStar; ++k) {
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
#pragma unroll
    for (int k = 0; k < kMaxStar; ++k) {
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
    typename St::L Lc = L[tl.c];
    typename St::L Ll[kMaxStar];
#pragma unroll
    for (int k = 0; k < kMaxStar; ++k)
        if (k < tl.depth) Ll[k] = L[tl.enc[k] & ~kCenterIsDst];
#pragma unroll
    for (int k = 0; k < kMaxStar; ++k)
        if (k < tl.depth) St::step_center(Lc, Ll[k], tl.enc[k] & kCenterIsDst, tl.x[k], tl.w[k]);
    typename St::X *px = slot_x + tl.base + lane;
#pragma unroll
    for (int k = 0; k < kMaxStar; ++k) {
        if (k < tl.depth) {
            px[k * kWave] = tl.x[k];
            L[tl.enc[k] & ~kCenterIsDst] = Ll[k];
        }
    }
    L[tl.c] = Lc;
}

// --------------------------------------------------- whole-GPU phase -----
constexpr int kPhaseBlock = 64;    // one tile per block: spread over many CUs

template <class St, bool kWeighted>
__global__ void __launch_bounds__(kPhaseBlock)
k_phase(PhaseDesc d, const int32_t *__restrict__ tile_center,
        const uint32_t *__restrict__ slot_leaf, typename St::X *__restrict__ slot_x,
        const float *__restrict__ slot_w, typename St::L *__restrict__ L) {
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t t = __builtin_amdgcn_readfirstlane(
        (int32_t)(blockIdx.x * (kPhaseBlock / kWave) + threadIdx.x / kWave));
    if (t >= d.T[0]) return;
    Tile<St, kWeighted> tl;
    load_tile(tl, d, t, lane, tile_center, slot_leaf, slot_x, slot_w);
    run_tile(tl, lane, slot_x, L);
}

// ----------------------------------------- single-workgroup phases -------
// The narrow phases after the whole-GPU ones run inside ONE workgroup, one
// after another, separated by workgroup barriers instead of kernel
// boundaries:
//  * middle phases: the node loads stay in global memory; all accesses come
//    from one CU, so they are coherent through its L1/L2 and a workgroup
//    barrier orders them (one CU's random-access rate, about one cache line
//    per clock, bounds this tier: it pays only for phases of a few hundred
//    edges);
//  * last phases: their nodes' loads are staged in LDS (with the tail's own
//    dummy entries) and written back at the end; an LDS-only barrier orders
//    them.
// Wave w owns tiles w, w + W, ... of every phase.  Each wave keeps two tile
// buffers: while it runs phase p from one, the other already receives its
// first tile of phase p+1 (leaf ids and fractions do not depend on phase p;
// only the loads do).  The buffers alternate, so no register copy forces
// the prefetch to complete.  Phase descriptors are staged in LDS.
constexpr int kTailBlock = 512;
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
    for (int k = 0; k < kMaxStar; ++k) d.T[k] = __builtin_amdgcn_readlane(v, 3 + k);
    d.pad = 0;
    return d;
}

// Runs the wave's tiles of one phase: the first from the prefetched buffer,
// any further ones (phase wider than the workgroup) loaded into that same
// buffer afterwards.
template <class St, bool kWeighted, class LPtr>
__device__ __forceinline__ void serial_phase(Tile<St, kWeighted> &tl, const PhaseDesc &d, int wave,
                                             int lane, const int32_t *__restrict__ tile_center,
                                             const uint32_t *__restrict__ slot_leaf,
                                             typename St::X *__restrict__ slot_x,
                                             const float *__restrict__ slot_w, LPtr L) {
    if (wave >= d.T[0]) return;
    run_tile(tl, lane, slot_x, L);
    for (int32_t t = wave + kTailWaves; t < d.T[0]; t += kTailWaves) {
        load_tile(tl, d, t, lane, tile_center, slot_leaf, slot_x, slot_w);
        run_tile(tl, lane, slot_x, L);
    }
}

template <bool kLds>
__device__ __forceinline__ void serial_barrier() {
    if (kLds) lds_barrier();
    else __syncthreads();
}

// The phase loop of a single-workgroup tier: phases [0, nph) whose
// descriptors are staged at sd, node loads at L (LDS or global).
template <class St, bool kWeighted, bool kLds, class LPtr>
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
        serial_phase(ta, da, wave, lane, tile_center, slot_leaf, slot_x, slot_w, L);
        serial_barrier<kLds>();
        if (!has_b) break;
        if (p + 2 < nph) {
            da = desc_from_lds(sd, p + 2, lane);
            if (wave < da.T[0]) load_tile(ta, da, wave, lane, tile_center, slot_leaf, slot_x, slot_w);
        }
        serial_phase(tb, db, wave, lane, tile_center, slot_leaf, slot_x, slot_w, L);
        serial_barrier<kLds>();
    }
}

__device__ __forceinline__ void stage_descs(int32_t nph, const PhaseDesc *descs, PhaseDesc *sd) {
    const int32_t *src = reinterpret_cast<const int32_t *>(descs);
    int32_t *dst = reinterpret_cast<int32_t *>(sd);
    const int32_t words = nph * (int32_t)(sizeof(PhaseDesc) / 4);
    for (int32_t i = threadIdx.x; i < words; i += blockDim.x) dst[i] = src[i];
}

template <class St, bool kWeighted, bool kLds>
__global__ void __launch_bounds__(kTailBlock)
k_serial(int32_t nph, const PhaseDesc *__restrict__ descs, const int32_t *__restrict__ tile_center,
         const uint32_t *__restrict__ slot_leaf, typename St::X *__restrict__ slot_x,
         const float *__restrict__ slot_w, const int32_t *__restrict__ tail_nodes, int32_t ntail,
         typename St::L *__restrict__ Lg) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    PhaseDesc *sd = reinterpret_cast<PhaseDesc *>(lds_raw);
    typename St::L *sL = reinterpret_cast<typename St::L *>(lds_raw + tail_desc_bytes(nph));
    typename St::L *L = kLds ? sL : Lg;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    stage_descs(nph, descs, sd);
    if (kLds) {
        constexpr int U = 8;   // eight gathers in flight per thread
        for (int32_t i0 = threadIdx.x; i0 < ntail; i0 += U * kTailBlock) {
            typename St::L v[U];
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int32_t i = i0 + j * kTailBlock;
                if (i < ntail) v[j] = Lg[tail_nodes[i]];
            }
#pragma unroll
            for (int j = 0; j < U; ++j) {
                const int32_t i = i0 + j * kTailBlock;
                if (i < ntail) sL[i] = v[j];
            }
        }
        if (threadIdx.x == 0) {
            sL[ntail] = St::from_f64(0.0);      // dummy center of empty lanes
            sL[ntail + 1] = St::infinite();     // dummy leaf of padding rows
        }
    }
    __syncthreads();
    run_phases<St, kWeighted, kLds>(nph, sd, wave, lane, tile_center, slot_leaf, slot_x, slot_w, L);
    if (kLds) {
        for (int32_t i = threadIdx.x; i < ntail; i += kTailBlock) Lg[tail_nodes[i]] = sL[i];
    }
}

// ------------------------------------------------------- batched graphs --
// Many independent unweighted graphs in one persistent launch: each
// workgroup takes the next graph from a queue (graphs ordered by edge count,
// largest first), builds its loads in LDS (deg / 2: a sum of halves, exact
// in any order), runs `sweeps` sweeps of the graph's phases from LDS, and
// writes the loads out.  Node ids of a graph are local (0..n_g-1); n_g and
// n_g + 1 are its dummy entries.
template <class St>
__global__ void __launch_bounds__(kTailBlock)
k_batch(int32_t G, const int32_t *__restrict__ order, unsigned *__restrict__ queue,
        const int64_t *__restrict__ node_ptr, const int64_t *__restrict__ edge_ptr,
        const int32_t *__restrict__ src, const int32_t *__restrict__ dst,
        const int64_t *__restrict__ desc_ptr, const PhaseDesc *__restrict__ descs,
        const int32_t *__restrict__ tile_center, const uint32_t *__restrict__ slot_leaf,
        typename St::X *__restrict__ slot_x, int32_t sweeps, double *__restrict__ Lout) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ int32_t s_graph;
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x / kWave);
    for (;;) {
        if (threadIdx.x == 0) {
            const unsigned k = atomicAdd(queue, 1u);
            s_graph = k < (unsigned)G ? order[k] : -1;
        }
        __syncthreads();
        const int32_t g = s_graph;
        if (g < 0) break;
        const int32_t n = (int32_t)(node_ptr[g + 1] - node_ptr[g]);
        const int64_t e0 = edge_ptr[g];
        const int64_t m = edge_ptr[g + 1] - e0;
        const int32_t nph = (int32_t)(desc_ptr[g + 1] - desc_ptr[g]);
        PhaseDesc *sd = reinterpret_cast<PhaseDesc *>(lds_raw);
        typename St::L *sL = reinterpret_cast<typename St::L *>(lds_raw + tail_desc_bytes(nph));
        double *cnt = reinterpret_cast<double *>(sL);   // degree halves, then loads in place
        stage_descs(nph, descs + desc_ptr[g], sd);
        // init: each edge adds one half to both ends (kept in FP64 first)
        for (int32_t u = threadIdx.x; u < n; u += kTailBlock) cnt[u] = 0.0;
        __syncthreads();
        for (int64_t e = threadIdx.x; e < m; e += kTailBlock) {
            atomicAdd(&cnt[src[e0 + e]], 0.5);
            atomicAdd(&cnt[dst[e0 + e]], 0.5);
        }
        __syncthreads();
        static_assert(sizeof(typename St::L) == sizeof(double), "loads converted in place");
        for (int32_t u = threadIdx.x; u < n; u += kTailBlock) {
            const double v = cnt[u];
            sL[u] = St::from_f64(v);
        }
        if (threadIdx.x == 0) {
            sL[n] = St::from_f64(0.0);
            sL[n + 1] = St::infinite();
        }
        __syncthreads();
        for (int32_t t = 0; t < sweeps; ++t)
            run_phases<St, false, true>(nph, sd, wave, lane, tile_center, slot_leaf, slot_x,
                                        nullptr, sL);
        __syncthreads();
        const int64_t n0 = node_ptr[g];
        for (int32_t u = threadIdx.x; u < n; u += kTailBlock) Lout[n0 + u] = St::to_f64(sL[u]);
        __syncthreads();   // LDS reuse by the next graph
    }
}

__global__ void k_zero_u32(unsigned *p) { *p = 0u; }

// ------------------------------------------------------------ statistics --
constexpr int kRedBlock = 256;

// FP64 loads recomputed from the fractions (f_e(src) = x, f_e(dst) = w - x);
// one wavefront per node, lanes stride over the row, fixed-order reduction
template <class St, bool kWeighted>
__global__ void __launch_bounds__(256) k_recompute(int32_t n, const int64_t *row_ptr,
                                                   const uint32_t *inc, const int64_t *edge_slot,
                                                   const typename St::X *slot_x, const float *w,
                                                   double *L64) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t u = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; u < n;
         u += waves) {
        double acc = 0.0;
        for (int64_t j = row_ptr[u] + lane; j < row_ptr[u + 1]; j += kWave) {
            uint32_t ent = inc[j];
            int64_t e = ent >> 1;
            double x = (double)slot_x[edge_slot[e]];
            double we = kWeighted ? (double)w[e] : 1.0;
            acc = acc + ((ent & 1) ? we - x : x);
        }
        for (int d = kWave / 2; d > 0; d >>= 1) acc = acc + __shfl_down(acc, d, kWave);
        if (lane == 0) L64[u] = acc;
    }
}

template <class St>
__global__ void k_loads_to_f64(int32_t n, const typename St::L *L, double *L64) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x)
        L64[u] = St::to_f64(L[u]);
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
                       void *L, hipStream_t s) {
        hipLaunchKernelGGL((k_init_loads<St, kW>), dim3(grid_for((int64_t)n + 2, 256)), dim3(256), 0, s, n,
                           row_ptr, inc, w, (typename St::L *)L);
    };
    fn.phase = [](const PhaseDesc &d, const int32_t *tile_center, const uint32_t *slot_leaf,
                  void *slot_x, const float *slot_w, void *L, hipStream_t s) {
        int32_t tiles = d.T[0];
        unsigned blocks = (unsigned)((tiles + (kPhaseBlock / kWave) - 1) / (kPhaseBlock / kWave));
        hipLaunchKernelGGL((k_phase<St, kW>), dim3(blocks), dim3(kPhaseBlock), 0, s, d,
                           tile_center, slot_leaf, (typename St::X *)slot_x, slot_w,
                           (typename St::L *)L);
    };
    fn.tail = [](int32_t nph, const PhaseDesc *descs, const int32_t *tile_center,
                 const uint32_t *slot_leaf, void *slot_x, const float *slot_w,
                 const int32_t *tail_nodes, int32_t ntail, void *L, hipStream_t s) {
        size_t lds = tail_desc_bytes(nph) + (size_t)(ntail + 2) * sizeof(typename St::L);
        hipLaunchKernelGGL((k_serial<St, kW, true>), dim3(1), dim3(kTailBlock), lds, s, nph, descs,
                           tile_center, slot_leaf, (typename St::X *)slot_x, slot_w, tail_nodes,
                           ntail, (typename St::L *)L);
    };
    fn.mid = [](int32_t nph, const PhaseDesc *descs, const int32_t *tile_center,
                const uint32_t *slot_leaf, void *slot_x, const float *slot_w, void *L,
                hipStream_t s) {
        size_t lds = tail_desc_bytes(nph);
        hipLaunchKernelGGL((k_serial<St, kW, false>), dim3(1), dim3(kTailBlock), lds, s, nph,
                           descs, tile_center, slot_leaf, (typename St::X *)slot_x, slot_w,
                           nullptr, 0, (typename St::L *)L);
    };
    fn.set_tail_lds = [](size_t bytes) {
        LOWD_HIP(hipFuncSetAttribute((const void *)k_serial<St, kW, true>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    };
    fn.set_mid_lds = [](size_t bytes) {
        LOWD_HIP(hipFuncSetAttribute((const void *)k_serial<St, kW, false>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    };
    fn.loads_f64 = [](int32_t n, const int64_t *row_ptr, const uint32_t *inc,
                      const int64_t *edge_slot, const void *slot_x, const float *w, const void *L,
                      double *L64, hipStream_t s) {
        if (St::kRecompute)
            hipLaunchKernelGGL((k_recompute<St, kW>), dim3(grid_for((int64_t)n * kWave, 256)),
                               dim3(256), 0, s, n, row_ptr, inc, edge_slot,
                               (const typename St::X *)slot_x, w, L64);
        else
            hipLaunchKernelGGL((k_loads_to_f64<St>), dim3(grid_for(n, 256)), dim3(256), 0, s, n,
                               (const typename St::L *)L, L64);
    };
    fn.read_x = [](int64_t m, const int64_t *edge_slot, const void *slot_x, double *x,
                   hipStream_t s) {
        hipLaunchKernelGGL((k_read_x<St>), dim3(grid_for(m, 256)), dim3(256), 0, s, m, edge_slot,
                           (const typename St::X *)slot_x, x);
    };
    fn.read_loads = [](int32_t n, const void *L, double *out, hipStream_t s) {
        hipLaunchKernelGGL((k_loads_to_f64<St>), dim3(grid_for(n, 256)), dim3(256), 0, s, n,
                           (const typename St::L *)L, out);
    };
    fn.batch = [](int32_t G, const int32_t *order, unsigned *queue, const int64_t *node_ptr,
                  const int64_t *edge_ptr, const int32_t *src, const int32_t *dst,
                  const int64_t *desc_ptr, const PhaseDesc *descs, const int32_t *tile_center,
                  const uint32_t *slot_leaf, void *slot_x, int32_t sweeps, double *Lout,
                  size_t lds, int32_t blocks, hipStream_t s) {
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, s, queue);
        hipLaunchKernelGGL((k_batch<St>), dim3((unsigned)blocks), dim3(kTailBlock), lds, s, G,
                           order, queue, node_ptr, edge_ptr, src, dst, desc_ptr, descs,
                           tile_center, slot_leaf, (typename St::X *)slot_x, sweeps, Lout);
    };
    fn.set_batch_lds = [](size_t bytes) {
        LOWD_HIP(hipFuncSetAttribute((const void *)k_batch<St>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    };
    fn.x_bytes = sizeof(typename St::X);
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

void launch_stats(int64_t n, const double *L64, double *partial, int32_t nb, double *out,
                  hipStream_t s) {
    hipLaunchKernelGGL(k_stats_partial, dim3((unsigned)nb), dim3(kRedBlock), 0, s, n, L64, partial);
    hipLaunchKernelGGL(k_stats_final, dim3(1), dim3(kRedBlock), 0, s, nb, partial, out);
}

}  // namespace lowd
