// k_greedy.hip -- greedy peeling (the appendix's Algorithm 3) on the GPU,
// exactly as its sequential definition: starting from S = V and S* = V,
// remove a node of minimum degree in S (ties: the smallest id) with its
// edges, and replace S* by S whenever rho(S) > rho(S*).  It is the second
// solver that Algorithm 2's pruning can feed (the plug-in DSPSolver).
//
// The removals are inherently one at a time, so one workgroup runs them all
// while the device memory holds the bucket structure: for every degree d a
// bitset over the node ids (bit u set iff u is alive with degree d), and a
// summary bitset with one bit per 64-bit word that may be non-zero.  A step:
//   1. the lowest non-empty degree (a counter per degree; it drops by at
//      most one per step);
//   2. the smallest id in that bucket: the first summary word with a bit
//      set, then the first non-zero word under it (a stale summary word whose
//      words are all zero is cleared and the search repeats);
//   3. the node leaves its bucket; |E(S)| and |S| drop; S* is updated by an
//      exact comparison of densities;
//   4. every alive neighbour moves one bucket down (atomics on the words and
//      counters), all lanes of the workgroup in parallel.
// Summary bits are only set during step 4 and only cleared in step 2, when
// no other lane writes, so no node is ever lost from the search.
#include <stdint.h>

#include <algorithm>
#include <string>
#include <vector>

#include "lowd_internal.h"

namespace lowd {
namespace {

constexpr int kGreedyBlock = 1024;

__global__ void k_greedy_init(int32_t n, const int64_t *row_ptr, int32_t *deg, uint64_t *words,
                              uint64_t *summ, int32_t *count, int64_t W, int64_t S) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t d = row_ptr[u + 1] - row_ptr[u];
        deg[u] = (int32_t)d;
        atomicOr((unsigned long long *)&words[d * W + (u >> 6)], 1ull << (u & 63));
        atomicOr((unsigned long long *)&summ[d * S + (u >> 12)], 1ull << ((u >> 6) & 63));
        atomicAdd(&count[d], 1);
    }
}

__device__ __forceinline__ int64_t block_min_i64(int64_t v, int64_t *lds) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    for (int d = kWave / 2; d > 0; d >>= 1) {
        const int64_t o = __shfl_down(v, d, kWave);
        v = o < v ? o : v;
    }
    if (lane == 0) lds[wave] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 1; k < kGreedyBlock / kWave; ++k) v = lds[k] < v ? lds[k] : v;
        lds[0] = v;
    }
    __syncthreads();
    const int64_t r = lds[0];
    __syncthreads();
    return r;
}

__global__ void __launch_bounds__(kGreedyBlock)
k_greedy(int32_t n, int64_t m, int32_t maxd, const int64_t *row_ptr, const uint32_t *inc,
         const int32_t *src, const int32_t *dst, int32_t *deg, uint64_t *words, uint64_t *summ,
         int32_t *count, int64_t W, int64_t S, int32_t *order, int64_t *rem_m, int64_t *best) {
    __shared__ int64_t lds[kGreedyBlock / kWave];
    __shared__ int32_t s_d, s_u;
    __shared__ int64_t s_sw;
    __shared__ int32_t s_blk;
    __shared__ int64_t s_M, s_N, s_bM, s_bN, s_bi;
    const int tid = threadIdx.x;
    if (tid == 0) {
        s_d = 0;
        s_M = m;
        s_N = n;
        s_bM = m;
        s_bN = n;
        s_bi = 0;
    }
    __syncthreads();
    for (int32_t step = 0; step < n; ++step) {
        // 1. the lowest non-empty degree
        if (tid == 0) {
            int32_t d = s_d;
            while (d < maxd && count[d] == 0) ++d;
            s_d = d;
        }
        __syncthreads();
        const int32_t d = s_d;
        uint64_t *wd = words + (int64_t)d * W;
        uint64_t *sd = summ + (int64_t)d * S;
        // 2. the smallest id in bucket d
        bool lost = false;
        for (;;) {
            int64_t first = INT64_MAX;
            for (int64_t s = tid; s < S; s += kGreedyBlock)
                if (sd[s] != 0) {
                    first = s;
                    break;
                }
            const int64_t sw = block_min_i64(first, lds);
            if (sw == INT64_MAX) {   // no candidate: the bucket invariant is broken
                lost = true;
                break;
            }
            if (tid < kWave) {
                const uint64_t sbits = sd[sw];
                const int64_t wi = sw * 64 + tid;
                const bool hit = ((sbits >> tid) & 1ull) && wi < W && wd[wi] != 0;
                const uint64_t mask = __ballot(hit);
                if (tid == 0) {
                    s_sw = sw;
                    s_blk = mask ? (int32_t)__builtin_ctzll(mask) : -1;
                    if (!mask) sd[sw] = 0;   // every word under it is empty
                }
            }
            __syncthreads();
            if (s_blk >= 0) break;
        }
        if (lost) {   // uniform: every lane saw the same reduction
            if (tid == 0) best[0] = -1;
            return;
        }
        // 3. remove the node
        if (tid == 0) {
            const int64_t wi = s_sw * 64 + s_blk;
            const uint64_t word = wd[wi];
            const int32_t u = (int32_t)(wi * 64 + __builtin_ctzll(word));
            wd[wi] = word & ~(1ull << (u & 63));
            count[d] -= 1;
            order[step] = u;
            s_u = u;
            s_M -= d;
            s_N -= 1;
            rem_m[step] = s_M;
            if (s_N > 0 && (__int128)s_M * s_bN > (__int128)s_bM * s_N) {
                s_bM = s_M;
                s_bN = s_N;
                s_bi = step + 1;
            }
            deg[u] = -1;
            s_d = d > 0 ? d - 1 : 0;
        }
        __syncthreads();
        // 4. its alive neighbours move one bucket down
        const int32_t u = s_u;
        for (int64_t j = row_ptr[u] + tid; j < row_ptr[u + 1]; j += kGreedyBlock) {
            const uint32_t ent = inc[j];
            const int64_t e = ent >> 1;
            const int32_t v = (ent & 1) ? src[e] : dst[e];
            const int32_t dv = deg[v];
            if (dv <= 0) continue;   // removed (an alive neighbour of u has degree >= 1)
            deg[v] = dv - 1;
            const uint64_t bit = 1ull << (v & 63);
            atomicAnd((unsigned long long *)&words[(int64_t)dv * W + (v >> 6)], ~bit);
            atomicOr((unsigned long long *)&words[(int64_t)(dv - 1) * W + (v >> 6)], bit);
            atomicOr((unsigned long long *)&summ[(int64_t)(dv - 1) * S + (v >> 12)],
                     1ull << ((v >> 6) & 63));
            atomicSub(&count[dv], 1);
            atomicAdd(&count[dv - 1], 1);
        }
        __syncthreads();
    }
    if (tid == 0) best[0] = s_bi;
}

__global__ void k_greedy_in_set(int32_t n, const int32_t *order, int64_t best_i, uint8_t *in_set) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        in_set[order[i]] = i >= best_i ? 1 : 0;
}

}  // namespace

int64_t greedy_peel(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, int32_t *order,
                    int64_t *rem_m, uint8_t *in_set, int64_t max_bytes, hipStream_t s) {
    Csr csr;
    build_incidence(n, m, src, dst, csr, s);
    // the largest degree sizes the buckets
    std::vector<int64_t> rp((size_t)n + 1);
    LOWD_HIP(hipMemcpyAsync(rp.data(), csr.row_ptr.p, rp.size() * sizeof(int64_t),
                            hipMemcpyDeviceToHost, s));
    LOWD_HIP(hipStreamSynchronize(s));
    int64_t maxd = 0;
    for (int32_t u = 0; u < n; ++u) maxd = std::max(maxd, rp[(size_t)u + 1] - rp[(size_t)u]);
    const int64_t W = ((int64_t)n + 63) / 64, S = (W + 63) / 64;
    const int64_t bytes = (maxd + 1) * (W + S) * 8;
    if (bytes > max_bytes)
        fail(LOWD_E_UNSUPPORTED, "greedy peeling needs " + std::to_string(bytes >> 20) +
                     " MiB of bucket bitsets (degree range x nodes); prune the graph first");
    DBuf<uint64_t> words((size_t)((maxd + 1) * W)), summ((size_t)((maxd + 1) * S));
    DBuf<int32_t> deg((size_t)n), count((size_t)maxd + 1);
    DBuf<int64_t> best(1);
    LOWD_HIP(hipMemsetAsync(words.p, 0, words.bytes(), s));
    LOWD_HIP(hipMemsetAsync(summ.p, 0, summ.bytes(), s));
    LOWD_HIP(hipMemsetAsync(count.p, 0, count.bytes(), s));
    hipLaunchKernelGGL(k_greedy_init, dim3(grid_for(n, 256)), dim3(256), 0, s, n, csr.row_ptr.p,
                       deg.p, words.p, summ.p, count.p, W, S);
    hipLaunchKernelGGL(k_greedy, dim3(1), dim3(kGreedyBlock), 0, s, n, m, (int32_t)maxd,
                       csr.row_ptr.p, csr.inc.p, src, dst, deg.p, words.p, summ.p, count.p, W, S,
                       order, rem_m, best.p);
    int64_t bi = 0;
    LOWD_HIP(hipMemcpyAsync(&bi, best.p, sizeof(bi), hipMemcpyDeviceToHost, s));
    LOWD_HIP(hipStreamSynchronize(s));
    if (bi < 0) fail(LOWD_E_HIP, "greedy peeling lost track of a degree bucket");
    if (in_set)
        hipLaunchKernelGGL(k_greedy_in_set, dim3(grid_for(n, 256)), dim3(256), 0, s, n, order, bi,
                           in_set);
    LOWD_HIP(hipGetLastError());
    LOWD_HIP(hipStreamSynchronize(s));
    return bi;
}

}  // namespace lowd
