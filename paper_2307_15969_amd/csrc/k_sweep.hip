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
        slot_x[s] = St::half_weight(we);
        if (kWeighted) slot_w[s] = we;
    }
}

// l_u = sum of w_e / 2 over the edges at u, in ascending edge index
template <class St, bool kWeighted>
__global__ void k_init_loads(int32_t n, const int64_t *row_ptr, const uint32_t *inc,
                             const float *w, typename St::L *L) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j) {
            double we = kWeighted ? (double)w[inc[j] >> 1] : 1.0;
            acc = acc + we / 2.0;
        }
        L[u] = St::from_f64(acc);
    }
}

// ------------------------------------------------------------ one tile ---
// The lane's star: center c (load in a register), leaves in rows 0..depth-1.
// Rows are read four at a time so the leaf loads of a group are in flight
// together; leaves of one star are distinct and belong to no other star of
// the phase, so a prefetched leaf load cannot be stale.
template <class St, bool kWeighted, class LPtr>
__device__ __forceinline__ void run_star(int32_t c, int64_t base, int32_t depth, int lane,
                                         const uint32_t *__restrict__ slot_leaf,
                                         typename St::X *__restrict__ slot_x,
                                         const float *__restrict__ slot_w, LPtr L) {
    typename St::L Lc = L[c];
    constexpr int G = 4;
    for (int k0 = 0; k0 < depth; k0 += G) {
        uint32_t enc[G];
        typename St::X xv[G];
        float wv[G];
        typename St::L Ll[G];
#pragma unroll
        for (int j = 0; j < G; ++j) {
            int64_t s = base + (int64_t)(k0 + j) * kWave + lane;
            enc[j] = (k0 + j < depth) ? slot_leaf[s] : kLeafPad;
        }
#pragma unroll
        for (int j = 0; j < G; ++j) {
            int64_t s = base + (int64_t)(k0 + j) * kWave + lane;
            if (enc[j] != kLeafPad) {
                xv[j] = slot_x[s];
                wv[j] = kWeighted ? slot_w[s] : 1.0f;
                Ll[j] = L[enc[j] & ~kCenterIsDst];
            }
        }
#pragma unroll
        for (int j = 0; j < G; ++j) {
            if (enc[j] == kLeafPad) break;
            int64_t s = base + (int64_t)(k0 + j) * kWave + lane;
            if (enc[j] & kCenterIsDst) St::step(Ll[j], Lc, xv[j], wv[j]);   // u = leaf
            else St::step(Lc, Ll[j], xv[j], wv[j]);                          // u = center
            slot_x[s] = xv[j];
            L[enc[j] & ~kCenterIsDst] = Ll[j];
        }
        if (enc[G - 1] == kLeafPad) break;
    }
    L[c] = Lc;
}

// --------------------------------------------------- whole-GPU phase -----
constexpr int kPhaseBlock = 256;   // four tiles per block

template <class St, bool kWeighted>
__global__ void __launch_bounds__(kPhaseBlock)
k_phase(int32_t tile_begin, int32_t tile_end, const int32_t *__restrict__ tile_center,
        const int64_t *__restrict__ tile_base, const int32_t *__restrict__ tile_depth,
        const uint32_t *__restrict__ slot_leaf, typename St::X *__restrict__ slot_x,
        const float *__restrict__ slot_w, typename St::L *__restrict__ L) {
    const int lane = threadIdx.x & (kWave - 1);
    const int32_t tile = tile_begin + (int32_t)(blockIdx.x * (kPhaseBlock / kWave) + threadIdx.x / kWave);
    if (tile >= tile_end) return;
    const int32_t c = tile_center[(int64_t)tile * kWave + lane];
    if (c < 0) return;
    run_star<St, kWeighted>(c, tile_base[tile], tile_depth[tile], lane, slot_leaf, slot_x, slot_w,
                            L);
}

// ----------------------------------------- LDS-resident last phases ------
constexpr int kTailBlock = 1024;

template <class St, bool kWeighted>
__global__ void __launch_bounds__(kTailBlock)
k_tail(int32_t nph, const int32_t *__restrict__ ph_tile_ptr, const int32_t *__restrict__ tile_center,
       const int64_t *__restrict__ tile_base, const int32_t *__restrict__ tile_depth,
       const uint32_t *__restrict__ slot_leaf, typename St::X *__restrict__ slot_x,
       const float *__restrict__ slot_w, const int32_t *__restrict__ tail_nodes, int32_t ntail,
       typename St::L *__restrict__ L) {
    extern __shared__ unsigned char lds_raw[];
    typename St::L *sL = reinterpret_cast<typename St::L *>(lds_raw);
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    constexpr int kWaves = kTailBlock / kWave;
    for (int32_t i = threadIdx.x; i < ntail; i += kTailBlock) sL[i] = L[tail_nodes[i]];
    __syncthreads();
    for (int32_t p = 0; p < nph; ++p) {
        const int32_t t0 = ph_tile_ptr[p], t1 = ph_tile_ptr[p + 1];
        for (int32_t t = t0 + wave; t < t1; t += kWaves) {
            const int32_t c = tile_center[(int64_t)t * kWave + lane];
            if (c >= 0)
                run_star<St, kWeighted>(c, tile_base[t], tile_depth[t], lane, slot_leaf, slot_x,
                                        slot_w, sL);
        }
        __syncthreads();
    }
    for (int32_t i = threadIdx.x; i < ntail; i += kTailBlock) L[tail_nodes[i]] = sL[i];
}

// ------------------------------------------------------------ statistics --
constexpr int kRedBlock = 256;

// FP64 loads recomputed from the fractions (f_e(src) = x, f_e(dst) = w - x)
template <class St, bool kWeighted>
__global__ void k_recompute(int32_t n, const int64_t *row_ptr, const uint32_t *inc,
                            const int64_t *edge_slot, const typename St::X *slot_x,
                            const float *w, double *L64) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x) {
        double acc = 0.0;
        for (int64_t j = row_ptr[u]; j < row_ptr[u + 1]; ++j) {
            uint32_t ent = inc[j];
            int64_t e = ent >> 1;
            double x = (double)slot_x[edge_slot[e]];
            double we = kWeighted ? (double)w[e] : 1.0;
            acc = acc + ((ent & 1) ? we - x : x);
        }
        L64[u] = acc;
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
        hipLaunchKernelGGL((k_init_loads<St, kW>), dim3(grid_for(n, 256)), dim3(256), 0, s, n,
                           row_ptr, inc, w, (typename St::L *)L);
    };
    fn.phase = [](int32_t t0, int32_t t1, const int32_t *tile_center, const int64_t *tile_base,
                  const int32_t *tile_depth, const uint32_t *slot_leaf, void *slot_x,
                  const float *slot_w, void *L, hipStream_t s) {
        int32_t tiles = t1 - t0;
        unsigned blocks = (unsigned)((tiles + (kPhaseBlock / kWave) - 1) / (kPhaseBlock / kWave));
        hipLaunchKernelGGL((k_phase<St, kW>), dim3(blocks), dim3(kPhaseBlock), 0, s, t0, t1,
                           tile_center, tile_base, tile_depth, slot_leaf,
                           (typename St::X *)slot_x, slot_w, (typename St::L *)L);
    };
    fn.tail = [](int32_t nph, const int32_t *ph_tile_ptr, const int32_t *tile_center,
                 const int64_t *tile_base, const int32_t *tile_depth, const uint32_t *slot_leaf,
                 void *slot_x, const float *slot_w, const int32_t *tail_nodes, int32_t ntail,
                 void *L, hipStream_t s) {
        size_t lds = (size_t)ntail * sizeof(typename St::L);
        hipLaunchKernelGGL((k_tail<St, kW>), dim3(1), dim3(kTailBlock), lds, s, nph, ph_tile_ptr,
                           tile_center, tile_base, tile_depth, slot_leaf,
                           (typename St::X *)slot_x, slot_w, tail_nodes, ntail,
                           (typename St::L *)L);
    };
    fn.set_tail_lds = [](size_t bytes) {
        LOWD_HIP(hipFuncSetAttribute((const void *)k_tail<St, kW>,
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    };
    fn.loads_f64 = [](int32_t n, const int64_t *row_ptr, const uint32_t *inc,
                      const int64_t *edge_slot, const void *slot_x, const float *w, const void *L,
                      double *L64, hipStream_t s) {
        if (St::kRecompute)
            hipLaunchKernelGGL((k_recompute<St, kW>), dim3(grid_for(n, 256)), dim3(256), 0, s, n,
                               row_ptr, inc, edge_slot, (const typename St::X *)slot_x, w, L64);
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
