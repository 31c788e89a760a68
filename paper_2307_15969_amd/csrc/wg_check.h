// wg_check.h -- the convergence check of one graph by one workgroup, for
// the batched solve: Section III-B's dual bound D = max load and Algorithm
// 1's extraction (sort the nodes by load, remove them one by one, keep the
// densest remaining set), with no kernel boundary and no host round trip.
//
// The graph's nodes are n0 .. n0+n-1 of the batch; the scratch arrays are
// the batch's, indexed by those global ids (each graph owns its slice, so
// workgroups never share an element).  Global scratch stays in the CU's L1
// and the L2 for a graph of a few thousand nodes; the workgroup barriers
// order it (all waves of a workgroup run on one CU).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lowd_internal.h"

namespace lowd {

constexpr int kSortDigits = 256;

template <int W>
struct WgCheckLds {
    uint32_t hw[W][kSortDigits];   // per-wave digit counts, then write offsets
    uint32_t tot[kSortDigits];     // digit totals, then their exclusive scan
    int64_t wsum[W];               // wave totals of a scan
    double dmax[W];
    int64_t bi[W], bw[W];          // per-wave best prefix
    int32_t skip;
};

// static LDS of the checks at the widest workgroup (16 waves), which the
// batch's dynamic LDS must leave room for
constexpr size_t kWgCheckLdsMax = sizeof(WgCheckLds<16>) + 64;

// order-preserving map of an FP64 value onto uint64 (-0 folded onto +0)
__device__ inline uint64_t wg_sortable(double v) {
    v = v + 0.0;
    const uint64_t b = __builtin_bit_cast(uint64_t, v);
    return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}

template <class T>
__device__ inline T wg_shfl_up(T v, int d) {
    const uint64_t u = __builtin_bit_cast(uint64_t, v);
    int lo = (int)(uint32_t)u, hi = (int)(uint32_t)(u >> 32);
    lo = __shfl_up(lo, d, kWave);
    hi = __shfl_up(hi, d, kWave);
    return __builtin_bit_cast(T, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ inline int64_t wave_incl_scan_i64(int64_t v, int lane) {
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const int64_t y = wg_shfl_up(v, d);
        if (lane >= d) v += y;
    }
    return v;
}

// Inclusive scan over the workgroup (W waves, threads in order); *total =
// the workgroup's sum.  Contains two barriers.
template <int W>
__device__ inline int64_t wg_incl_scan(int64_t v, WgCheckLds<W> &ls, int64_t *total) {
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int64_t inc = wave_incl_scan_i64(v, lane);
    if (lane == kWave - 1) ls.wsum[wave] = inc;
    __syncthreads();
    int64_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < W; ++k) {
        const int64_t t = ls.wsum[k];
        before += k < wave ? t : 0;
        all += t;
    }
    __syncthreads();
    *total = all;
    return inc + before;
}

// Largest value over the workgroup (every thread gets it).
template <int W>
__device__ inline double wg_max(double v, WgCheckLds<W> &ls) {
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    for (int d = kWave / 2; d > 0; d >>= 1) {
        const double o = __shfl_down(v, d, kWave);
        v = o > v ? o : v;
    }
    if (lane == 0) ls.dmax[wave] = v;
    __syncthreads();
    double r = ls.dmax[0];
#pragma unroll
    for (int k = 1; k < W; ++k) r = ls.dmax[k] > r ? ls.dmax[k] : r;
    __syncthreads();
    return r;
}

// Stable LSD radix sort of n (key, id) pairs by key, 8-bit digits, by one
// workgroup: wave w owns the contiguous range [n w / W, n (w+1) / W) of the
// current order; per digit pass it counts its range's digits, the
// digit-major exclusive scan over (digit, wave) gives every wave its write
// offsets, and the wave writes its range in order, ranking equal digits
// among its lanes with eight ballots.  A pass whose digit is the same for
// every key leaves the order as it is and is skipped.  Returns true when the
// result is in (kb, ib), false when in (ka, ia).
template <int W>
__device__ bool wg_radix_sort(uint64_t *ka, uint32_t *ia, uint64_t *kb, uint32_t *ib, int32_t n,
                              WgCheckLds<W> &ls) {
    static_assert(W * kWave >= kSortDigits, "a thread per digit");
    constexpr int kGroup = 4;   // chunks of 64 keys loaded before they are used
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    const int32_t lo = (int32_t)((int64_t)n * wave / W);
    const int32_t hi = (int32_t)((int64_t)n * (wave + 1) / W);
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    uint64_t *kin = ka, *kout = kb;
    uint32_t *iin = ia, *iout = ib;
    if (tid == 0) ls.skip = 0;
    __syncthreads();
    for (int shift = 0; shift < 64; shift += 8) {
        for (int d = lane; d < kSortDigits; d += kWave) ls.hw[wave][d] = 0u;
        for (int32_t c0 = lo; c0 < hi; c0 += kGroup * kWave) {
            uint64_t kk[kGroup];
#pragma unroll
            for (int j = 0; j < kGroup; ++j) {
                const int32_t i = c0 + j * kWave + lane;
                kk[j] = i < hi ? kin[i] : 0ull;
            }
#pragma unroll
            for (int j = 0; j < kGroup; ++j)
                if (c0 + j * kWave + lane < hi)
                    count_digit(ls.hw[wave], (uint32_t)(kk[j] >> shift) & (kSortDigits - 1));
        }
        __syncthreads();
        if (tid < kSortDigits) {
            uint32_t t = 0;
#pragma unroll
            for (int w = 0; w < W; ++w) t += ls.hw[w][tid];
            ls.tot[tid] = t;
            if (t == (uint32_t)n) ls.skip = 1;
        }
        __syncthreads();
        const bool skip = ls.skip != 0;
        __syncthreads();
        if (skip) {
            if (tid == 0) ls.skip = 0;
            __syncthreads();
            continue;
        }
        {   // exclusive scan of the digit totals (threads 0..255 hold them)
            int64_t total;
            const int64_t v = tid < kSortDigits ? (int64_t)ls.tot[tid] : 0;
            const int64_t inc = wg_incl_scan<W>(v, ls, &total);
            if (tid < kSortDigits) {
                uint32_t run = (uint32_t)(inc - v);
#pragma unroll
                for (int w = 0; w < W; ++w) {
                    const uint32_t c = ls.hw[w][tid];
                    ls.hw[w][tid] = run;
                    run += c;
                }
            }
        }
        __syncthreads();
        for (int32_t c0 = lo; c0 < hi; c0 += kGroup * kWave) {
            uint64_t kk[kGroup];
            uint32_t ii[kGroup];
#pragma unroll
            for (int j = 0; j < kGroup; ++j) {
                const int32_t i = c0 + j * kWave + lane;
                kk[j] = i < hi ? kin[i] : 0ull;
                ii[j] = i < hi ? iin[i] : 0u;
            }
#pragma unroll
            for (int j = 0; j < kGroup; ++j) {
                if (c0 + j * kWave >= hi) break;   // uniform across the wave
                const bool valid = c0 + j * kWave + lane < hi;
                const uint32_t d = (uint32_t)(kk[j] >> shift) & (kSortDigits - 1);
                uint64_t same = __ballot(valid);
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    const bool bit = (d >> b) & 1u;
                    const uint64_t ones = __ballot(valid && bit);
                    same &= bit ? ones : ~ones;
                }
                const uint32_t rank = (uint32_t)__popcll(same & lt);
                const uint32_t base = ls.hw[wave][d];
                if (valid) {
                    kout[base + rank] = kk[j];
                    iout[base + rank] = ii[j];
                }
                // every lane has read its digit's offset (one instruction
                // for the wave, LDS accesses of a wave in order) before the
                // first lane of each digit moves it on
                if (valid && rank == 0) ls.hw[wave][d] = base + (uint32_t)__popcll(same);
            }
        }
        __syncthreads();
        uint64_t *tk = kin;
        kin = kout;
        kout = tk;
        uint32_t *ti = iin;
        iin = iout;
        iout = ti;
    }
    return kin == kb;
}

// The densest removal prefix of the sorted order (Algorithm 1's extraction)
// from hist[p] = the number of edges whose lower-positioned endpoint sits at
// position p: W(S_i) = sum_{p >= i} hist[p] for S_i = the nodes at
// positions i..n-1, and the best i maximises W(S_i) / (n - i), the smallest
// i (the largest set) among equal densities, compared exactly.  Every thread
// gets (best i, W at it).
__device__ inline bool wg_denser(int64_t wa, int64_t ia, int64_t wb, int64_t ib, int64_t n) {
    // is prefix ia (weight wa) preferred to prefix ib (weight wb)?
    if (ib < 0) return true;
    const __int128 l = (__int128)wa * (n - ib), r = (__int128)wb * (n - ia);
    return l > r || (l == r && ia < ib);
}

template <int W>
__device__ inline void wg_best_prefix(const int32_t *hist, int32_t n, WgCheckLds<W> &ls,
                                      int64_t *best_i, int64_t *best_w) {
    const int tid = threadIdx.x, lane = tid & (kWave - 1), wave = tid / kWave;
    int64_t carry = 0, bi = -1, bw = 0;
    for (int32_t c0 = 0; c0 < n; c0 += W * kWave) {   // uniform across the workgroup
        const int32_t k = c0 + tid;
        const int32_t i = n - 1 - k;                  // descending positions
        const int64_t h = k < n ? (int64_t)hist[i] : 0;
        int64_t total;
        const int64_t inc = wg_incl_scan<W>(h, ls, &total);
        if (k < n && wg_denser(carry + inc, i, bw, bi, n)) {
            bi = i;
            bw = carry + inc;
        }
        carry += total;
    }
    for (int d = kWave / 2; d > 0; d >>= 1) {
        const int64_t oi = __shfl_down(bi, d, kWave), ow = __shfl_down(bw, d, kWave);
        if (oi >= 0 && wg_denser(ow, oi, bw, bi, n)) {
            bi = oi;
            bw = ow;
        }
    }
    if (lane == 0) {
        ls.bi[wave] = bi;
        ls.bw[wave] = bw;
    }
    __syncthreads();
    int64_t ri = ls.bi[0], rw = ls.bw[0];
#pragma unroll
    for (int k = 1; k < W; ++k)
        if (ls.bi[k] >= 0 && wg_denser(ls.bw[k], ls.bi[k], rw, ri, n)) {
            ri = ls.bi[k];
            rw = ls.bw[k];
        }
    __syncthreads();
    *best_i = ri;
    *best_w = rw;
}

// Sweeps before the next check from the last two (sweeps, gap) records:
// the gap decays about geometrically, so they predict when it reaches tol;
// at most every, at least 1 (t0 < 0: fewer than two records).
__device__ inline int32_t wg_next_check(int32_t t0, double g0, int32_t t1, double g1, double tol,
                                        int32_t every) {
    if (t0 >= 0 && g1 > 0.0 && g1 < g0 && t1 > t0 && g1 > tol) {
        const double rate = pow(g1 / g0, 1.0 / (double)(t1 - t0));
        if (rate < 1.0) {
            const double k = ceil(log(tol / g1) / log(rate));
            if (k < (double)every) return k > 1.0 ? (int32_t)k : 1;
        }
    }
    return every;
}

}  // namespace lowd
