// k_scan.hip -- device-wide exclusive scan (int64) and stable LSD radix sort
// of (key, value) pairs, written for 64-lane wavefronts.
//
// Scan: reduce-then-scan in three launches; inside a block every wavefront
// scans its 64 lanes with shuffles and the wave totals are scanned in LDS.
// Radix sort: 8-bit digits; per block an LDS digit histogram, one global
// exclusive scan of the digit-major block histograms, then a stable scatter
// in which every wavefront ranks its keys among equal digits with eight
// ballots (the lanes whose digit matches in all eight bits).  Large inputs
// stage the ranked keys in LDS and write each digit's run contiguously.
#include <utility>

#include "lowd_internal.h"

namespace lowd {
namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

// shuffle of an 8- or 16-byte value, 32 bits at a time
template <class T>
__device__ inline T shfl_up_64(T v, int d) {
    static_assert(sizeof(T) == 8 || sizeof(T) == 16, "8- or 16-byte values");
    struct Words {
        int w[sizeof(T) / 4];
    };
    Words x = __builtin_bit_cast(Words, v);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k) x.w[k] = __shfl_up(x.w[k], d, kWave);
    return __builtin_bit_cast(T, x);
}

// inclusive scan over the 64 lanes of a wavefront
template <class T>
__device__ inline T wave_inclusive_scan(T v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        T y = shfl_up_64(v, d);
        if (lane >= d) v = v + y;
    }
    return v;
}

// exclusive scan over the block; returns the block total in *total
template <class T>
__device__ inline T block_exclusive_scan(T v, T *lds_waves, T *total) {
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const int nwaves = blockDim.x / kWave;
    T inc = wave_inclusive_scan(v);
    if (lane == kWave - 1) lds_waves[wave] = inc;
    __syncthreads();
    if (wave == 0) {
        T t = lane < nwaves ? lds_waves[lane] : (T)0;
        T ti = wave_inclusive_scan(t);
        if (lane < nwaves) lds_waves[lane] = ti - t;   // exclusive wave offsets
        if (lane == nwaves - 1) lds_waves[kWave] = ti;  // block total
    }
    __syncthreads();
    T r = (inc - v) + lds_waves[wave];
    *total = lds_waves[kWave];
    __syncthreads();
    return r;
}

template <class T>
__global__ void __launch_bounds__(kScanBlock) k_scan_reduce(const T *in, int64_t n, T *partial) {
    __shared__ T lds[kWave + 1];
    int64_t base = (int64_t)blockIdx.x * kScanTile;
    T s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + (int64_t)k * kScanBlock + threadIdx.x;
        if (i < n) s = s + in[i];
    }
    T tot;
    block_exclusive_scan(s, lds, &tot);
    if (threadIdx.x == 0) partial[blockIdx.x] = tot;
}

// single block: exclusive scan of `partial` in place, total to *total
template <class T>
__global__ void __launch_bounds__(kScanBlock) k_scan_partials(T *partial, int64_t nb, T *total) {
    __shared__ T lds[kWave + 1];
    T carry = 0;
    for (int64_t base = 0; base < nb; base += kScanBlock) {
        int64_t i = base + threadIdx.x;
        T v = i < nb ? partial[i] : (T)0;
        T tot;
        T ex = block_exclusive_scan(v, lds, &tot);
        if (i < nb) partial[i] = ex + carry;
        carry = carry + tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

template <class T>
__global__ void __launch_bounds__(kScanBlock) k_scan_apply(const T *in, T *out, int64_t n,
                                                           const T *partial) {
    __shared__ T lds[kWave + 1];
    // each thread owns kScanItems consecutive items of the tile
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T v[kScanItems];
    T s = 0;
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        v[k] = i < n ? in[i] : (T)0;
        s = s + v[k];
    }
    T tot;
    T ex = block_exclusive_scan(s, lds, &tot) + partial[blockIdx.x];
    for (int k = 0; k < kScanItems; ++k) {
        int64_t i = base + k;
        if (i < n) out[i] = ex;
        ex = ex + v[k];
    }
}


// ------------------------------------------------------------ radix sort --
// A block sorts a chunk of `tiles` tiles of 256 keys per pass.  The chunk
// is sized to the input so that about kRadixTargetBlocks blocks share it
// (a fixed 64-tile chunk left 1M keys to 64 blocks on 256 CUs), at most
// kRadixMaxTiles tiles: larger inputs get more blocks instead.
constexpr int kRadixBlock = 256;
constexpr int64_t kRadixMaxTiles = 64;
constexpr int64_t kRadixTargetBlocks = 1024;
constexpr int kDigits = 256;
inline int64_t radix_tiles(int64_t n) {
    const int64_t per = kRadixTargetBlocks * kRadixBlock;
    const int64_t t = (n + per - 1) / per;
    return t < 1 ? 1 : (t > kRadixMaxTiles ? kRadixMaxTiles : t);
}

// A block counts the digits of its chunk (a multiple of 256 keys, so every
// 16-byte group of keys is aligned): 16 bytes of keys a lane per load, two
// loads in flight, the rest one key at a time.
template <class K>
__global__ void __launch_bounds__(kRadixBlock) k_radix_hist(const K *keys, int64_t n, int shift,
                                                            int64_t *blockhist, int64_t nb,
                                                            int64_t chunk) {
    constexpr int kV = 16 / sizeof(K);   // keys per 16-byte load
    struct alignas(16) Vec {
        K k[kV];
    };
    __shared__ uint32_t h[kDigits];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * chunk;
    const int64_t end = base + chunk < n ? base + chunk : n;
    constexpr int64_t kStep = 2 * kV * kRadixBlock;
    const int64_t vend = base + (end - base) / kStep * kStep;
    for (int64_t i = base + (int64_t)threadIdx.x * kV; i < vend; i += kStep) {
        const Vec a = *(const Vec *)(keys + i);
        const Vec b = *(const Vec *)(keys + i + kV * kRadixBlock);
#pragma unroll
        for (int q = 0; q < kV; ++q) {
            count_digit(h, (uint32_t)(a.k[q] >> shift) & (kDigits - 1));
            count_digit(h, (uint32_t)(b.k[q] >> shift) & (kDigits - 1));
        }
    }
    for (int64_t i = vend + threadIdx.x; i < end; i += kRadixBlock)
        count_digit(h, (uint32_t)(keys[i] >> shift) & (kDigits - 1));
    __syncthreads();
    blockhist[(int64_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// The scatter stages rounds of tiles in LDS in digit order, then writes
// every digit's run of the round to consecutive addresses: a tile's 256 keys
// written straight out land on up to 256 scattered lines, a round's runs
// average 16 keys per digit at 16 tiles (4,096 keys).  Rounds of 32 tiles
// (64 KB of LDS, two blocks a CU) measured faster for 8-byte keys alone
// (2 passes over 260M keys: 3.0 -> 2.8 ms) and slower for 4-byte keys with
// values (3 passes over 520M pairs: 9.4 -> 10.7 ms), so only the former
// take them.  Within a round wave w owns the contiguous quarter
// [w R/4, (w+1) R/4) of the keys: it counts its digits in a row of LDS
// counters of its own, one scan over (digit, wave) in that order gives every
// wave the first position of each digit, and the wave places its keys chunk
// by chunk in key order, ranking equal digits among its lanes with eight
// ballots and moving its own counters on.  Keys keep their order within a
// digit, so the permutation is the stable one.
template <class K, bool kVals>
constexpr int radix_round_tiles() {
    return sizeof(K) == 8 && !kVals ? 32 : 16;
}

template <class K, bool kVals>
__global__ void __launch_bounds__(kRadixBlock) k_radix_scatter_staged(const K *keys, const uint32_t *vals,
                                                               K *keys_out, uint32_t *vals_out,
                                                               int64_t n, int shift,
                                                               const int64_t *offsets,
                                                               int64_t nb, int64_t tiles) {
    constexpr int kWaves = kRadixBlock / kWave;
    constexpr int kRound = radix_round_tiles<K, kVals>() * kRadixBlock;   // keys staged at a time
    constexpr int kChunks = kRound / kRadixBlock;             // 64-key chunks a wave owns
    __shared__ int64_t running[kDigits];         // next global position of each digit
    __shared__ int64_t scan_lds[kWave + 1];
    __shared__ uint32_t cnt[kDigits];            // this round's keys per digit
    __shared__ uint32_t start[kDigits];          // their first local position
    __shared__ uint32_t wpos[kWaves][kDigits];   // a wave's digit counts, then its next positions
    __shared__ K skey[kRound];
    __shared__ uint32_t sval[kVals ? kRound : 1];
    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int wave = tid / kWave;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    running[tid] = offsets[(int64_t)tid * nb + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * tiles * kRadixBlock;
    const int64_t end = base + tiles * kRadixBlock < n ? base + tiles * kRadixBlock : n;
    for (int64_t r0 = base; r0 < end; r0 += kRound) {   // uniform across the block
        const int64_t r1 = r0 + kRound < end ? r0 + kRound : end;
        // this wave's quarter of the round, 64 keys a chunk in key order
        const int64_t lo = r0 + (int64_t)wave * (kRound / kWaves);
        const int64_t hi = lo + kRound / kWaves < r1 ? lo + kRound / kWaves : r1;
        K kreg[kChunks];
        uint32_t vreg[kChunks];
        for (int d = lane; d < kDigits; d += kWave) wpos[wave][d] = 0u;
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            const int64_t i = lo + (int64_t)c * kWave + lane;
            kreg[c] = i < hi ? keys[i] : (K)0;
            vreg[c] = kVals && i < hi ? vals[i] : 0u;
        }
#pragma unroll
        for (int c = 0; c < kChunks; ++c)
            if (lo + (int64_t)c * kWave + lane < hi)
                count_digit(wpos[wave], (uint32_t)(kreg[c] >> shift) & (kDigits - 1));
        __syncthreads();
        {   // digit totals, their scan, and each wave's first position per digit
            uint32_t t = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) t += wpos[w][tid];
            cnt[tid] = t;
            int64_t tot;
            const uint32_t st = (uint32_t)block_exclusive_scan<int64_t>((int64_t)t, scan_lds, &tot);
            start[tid] = st;
            uint32_t run = st;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                const uint32_t c = wpos[w][tid];
                wpos[w][tid] = run;
                run += c;
            }
        }
        __syncthreads();
        // each wave places its keys in order; its counters are its own
#pragma unroll
        for (int c = 0; c < kChunks; ++c) {
            if (lo + (int64_t)c * kWave >= hi) break;   // uniform across the wave
            const bool valid = lo + (int64_t)c * kWave + lane < hi;
            const uint32_t d = (uint32_t)(kreg[c] >> shift) & (kDigits - 1);
            uint64_t same = __ballot(valid);
#pragma unroll
            for (int b = 0; b < 8; ++b) {
                const bool bit = (d >> b) & 1u;
                const uint64_t ones = __ballot(valid && bit);
                same &= bit ? ones : ~ones;
            }
            const uint32_t rank = (uint32_t)__popcll(same & lt_mask);
            const uint32_t p = wpos[wave][d];
            if (valid) {
                skey[p + rank] = kreg[c];
                if (kVals) sval[p + rank] = vreg[c];
            }
            // every lane has read its digit's position (one instruction for
            // the wave, a wave's LDS accesses in order) before the first lane
            // of each digit moves it on
            if (valid && rank == 0) wpos[wave][d] = p + (uint32_t)__popcll(same);
        }
        __syncthreads();
        // every digit's run to consecutive global positions
        const int64_t m = r1 - r0;
        for (int64_t j = tid; j < m; j += kRadixBlock) {
            const K key = skey[j];
            const uint32_t d = (uint32_t)(key >> shift) & (kDigits - 1);
            const int64_t dst = running[d] + (j - (int64_t)start[d]);
            keys_out[dst] = key;
            if (kVals) vals_out[dst] = sval[j];
        }
        __syncthreads();
        running[tid] += cnt[tid];
        __syncthreads();
    }
}

// Per-tile scatter: every tile's keys go straight to their places.  Used
// below kRadixStagedTiles tiles per block, where the staged kernel's LDS
// (two blocks per CU) costs more than its coalescing gains.
template <class K, bool kVals>
__global__ void __launch_bounds__(kRadixBlock) k_radix_scatter_tiles(const K *keys, const uint32_t *vals,
                                                               K *keys_out, uint32_t *vals_out,
                                                               int64_t n, int shift,
                                                               const int64_t *offsets,
                                                               int64_t nb, int64_t tiles) {
    constexpr int kWaves = kRadixBlock / kWave;
    __shared__ int64_t running[kDigits];
    __shared__ int32_t wave_cnt[kWaves][kDigits];
    __shared__ int64_t wave_off[kWaves][kDigits];
    const int lane = threadIdx.x & (kWave - 1);
    const int wave = threadIdx.x / kWave;
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    running[threadIdx.x] = offsets[(int64_t)threadIdx.x * nb + blockIdx.x];
    int64_t base = (int64_t)blockIdx.x * tiles * kRadixBlock;
    for (int64_t t = 0; t < tiles; ++t) {
        int64_t tile0 = base + (int64_t)t * kRadixBlock;
        if (tile0 >= n) break;                       // uniform across the block
        int64_t i = tile0 + threadIdx.x;
        bool valid = i < n;
        K key = valid ? keys[i] : (K)0;
        uint32_t val = kVals && valid ? vals[i] : 0u;
        uint32_t d = (uint32_t)(key >> shift) & (kDigits - 1);
        for (int k = 0; k < kWaves; ++k) wave_cnt[k][threadIdx.x] = 0;
        // lanes of this wave holding the same digit
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            bool bit = (d >> b) & 1u;
            uint64_t ones = __ballot(valid && bit);
            same &= bit ? ones : ~ones;
        }
        int rank = __popcll(same & lt_mask);
        __syncthreads();
        if (valid && rank == 0) wave_cnt[wave][d] = __popcll(same);
        __syncthreads();
        {   // one thread per digit: offsets of each wave's group, in wave order
            int dd = threadIdx.x;
            int64_t r = running[dd];
            for (int k = 0; k < kWaves; ++k) {
                wave_off[k][dd] = r;
                r += wave_cnt[k][dd];
            }
            running[dd] = r;
        }
        __syncthreads();
        if (valid) {
            int64_t dst = wave_off[wave][d] + rank;
            keys_out[dst] = key;
            if (kVals) vals_out[dst] = val;
        }
        __syncthreads();
    }
}

constexpr int64_t kRadixStagedTiles = 32;

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// vals (and vals_alt) may be NULL: the keys alone are sorted.
template <class K>
void radix_sort_impl(K *keys, uint32_t *vals, K *keys_alt, uint32_t *vals_alt, int64_t n, int bits,
                     void *tmp, size_t tmp_bytes, bool *result_in_alt, hipStream_t s) {
    *result_in_alt = false;
    if (n <= 1 || bits <= 0) return;
    const int64_t tiles = radix_tiles(n), chunk = tiles * kRadixBlock;
    int64_t nb = cdiv(n, chunk);
    int64_t nh = nb * kDigits;
    if (tmp_bytes < radix_sort_tmp_bytes(n)) fail(LOWD_E_ARG, "radix sort scratch too small");
    int64_t *hist = (int64_t *)tmp;
    int64_t *scan_tmp = hist + nh;
    size_t scan_bytes = tmp_bytes - (size_t)nh * sizeof(int64_t);
    K *kin = keys, *kout = keys_alt;
    uint32_t *vin = vals, *vout = vals_alt;
    bool in_alt = false;
    for (int shift = 0; shift < bits; shift += 8) {
        hipLaunchKernelGGL(k_radix_hist<K>, dim3((unsigned)nb), dim3(kRadixBlock), 0, s, kin, n,
                           shift, hist, nb, chunk);
        exclusive_scan_i64(hist, hist, nh, nullptr, scan_tmp, scan_bytes, s);
        if (tiles >= kRadixStagedTiles) {
            if (vals)
                hipLaunchKernelGGL((k_radix_scatter_staged<K, true>), dim3((unsigned)nb),
                                   dim3(kRadixBlock), 0, s, kin, vin, kout, vout, n, shift, hist,
                                   nb, tiles);
            else
                hipLaunchKernelGGL((k_radix_scatter_staged<K, false>), dim3((unsigned)nb),
                                   dim3(kRadixBlock), 0, s, kin, vin, kout, vout, n, shift, hist,
                                   nb, tiles);
        } else {
            if (vals)
                hipLaunchKernelGGL((k_radix_scatter_tiles<K, true>), dim3((unsigned)nb),
                                   dim3(kRadixBlock), 0, s, kin, vin, kout, vout, n, shift, hist,
                                   nb, tiles);
            else
                hipLaunchKernelGGL((k_radix_scatter_tiles<K, false>), dim3((unsigned)nb),
                                   dim3(kRadixBlock), 0, s, kin, vin, kout, vout, n, shift, hist,
                                   nb, tiles);
        }
        LOWD_HIP(hipGetLastError());
        std::swap(kin, kout);
        std::swap(vin, vout);
        in_alt = !in_alt;
    }
    *result_in_alt = in_alt;
}

// starts[d] = first position of digit d after a pass (the scanned block
// histograms hold it at [d][0]); starts[kDigits] = n
__global__ void k_digit_starts(const int64_t *hist, int64_t nb, int64_t n, int64_t *starts) {
    const int d = threadIdx.x;
    if (d < kDigits) starts[d] = hist[(int64_t)d * nb];
    else if (d == kDigits) starts[kDigits] = n;
}

}  // namespace

void radix_partition_u32(const uint32_t *keys, uint32_t *keys_out, int64_t n, int shift,
                         int64_t *starts, void *tmp, size_t tmp_bytes, hipStream_t s) {
    if (tmp_bytes < radix_sort_tmp_bytes(n)) fail(LOWD_E_ARG, "radix partition scratch too small");
    if (n <= 0) {
        LOWD_HIP(hipMemsetAsync(starts, 0, (kDigits + 1) * sizeof(int64_t), s));
        return;
    }
    const int64_t tiles = radix_tiles(n), chunk = tiles * kRadixBlock;
    const int64_t nb = cdiv(n, chunk), nh = nb * kDigits;
    int64_t *hist = (int64_t *)tmp;
    int64_t *scan_tmp = hist + nh;
    const size_t scan_bytes = tmp_bytes - (size_t)nh * sizeof(int64_t);
    hipLaunchKernelGGL(k_radix_hist<uint32_t>, dim3((unsigned)nb), dim3(kRadixBlock), 0, s, keys,
                       n, shift, hist, nb, chunk);
    exclusive_scan_i64(hist, hist, nh, nullptr, scan_tmp, scan_bytes, s);
    if (tiles >= kRadixStagedTiles)
        hipLaunchKernelGGL((k_radix_scatter_staged<uint32_t, false>), dim3((unsigned)nb),
                           dim3(kRadixBlock), 0, s, keys, nullptr, keys_out, nullptr, n, shift,
                           hist, nb, tiles);
    else
        hipLaunchKernelGGL((k_radix_scatter_tiles<uint32_t, false>), dim3((unsigned)nb),
                           dim3(kRadixBlock), 0, s, keys, nullptr, keys_out, nullptr, n, shift,
                           hist, nb, tiles);
    hipLaunchKernelGGL(k_digit_starts, dim3(1), dim3(kDigits + 1), 0, s, hist, nb, n, starts);
    LOWD_HIP(hipGetLastError());
}

// scratch of a scan of up to n values of up to 16 bytes
size_t exclusive_scan_tmp_bytes(int64_t n) {
    int64_t nb = cdiv(n > 0 ? n : 1, kScanTile);
    return (size_t)(nb + 1) * 16;
}

namespace {
template <class T>
void exclusive_scan_impl(const T *in, T *out, int64_t n, T *total_dev, void *tmp,
                         size_t tmp_bytes, hipStream_t s) {
    if (n <= 0) return;
    int64_t nb = cdiv(n, kScanTile);
    if (tmp_bytes < exclusive_scan_tmp_bytes(n)) fail(LOWD_E_ARG, "scan scratch too small");
    T *partial = (T *)tmp;
    hipLaunchKernelGGL(k_scan_reduce<T>, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, n,
                       partial);
    hipLaunchKernelGGL(k_scan_partials<T>, dim3(1), dim3(kScanBlock), 0, s, partial, nb,
                       total_dev);
    hipLaunchKernelGGL(k_scan_apply<T>, dim3((unsigned)nb), dim3(kScanBlock), 0, s, in, out, n,
                       partial);
    LOWD_HIP(hipGetLastError());
}
}  // namespace

void exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total_dev, void *tmp,
                        size_t tmp_bytes, hipStream_t s) {
    exclusive_scan_impl<int64_t>(in, out, n, total_dev, tmp, tmp_bytes, s);
}

void exclusive_scan_f64(const double *in, double *out, int64_t n, double *total_dev, void *tmp,
                        size_t tmp_bytes, hipStream_t s) {
    exclusive_scan_impl<double>(in, out, n, total_dev, tmp, tmp_bytes, s);
}

void exclusive_scan_u128(const u128 *in, u128 *out, int64_t n, u128 *total_dev, void *tmp,
                         size_t tmp_bytes, hipStream_t s) {
    exclusive_scan_impl<u128>(in, out, n, total_dev, tmp, tmp_bytes, s);
}

size_t radix_sort_tmp_bytes(int64_t n) {
    // enough for every n' <= n: below the tile cap a sort uses at most
    // min(kRadixTargetBlocks, n' / 256) blocks, at the cap n' / (64 * 256)
    const int64_t m = n > 0 ? n : 1;
    const int64_t small = cdiv(m, kRadixBlock) < kRadixTargetBlocks ? cdiv(m, kRadixBlock)
                                                                    : kRadixTargetBlocks;
    const int64_t big = cdiv(m, kRadixMaxTiles * kRadixBlock);
    const int64_t nb = small > big ? small : big;
    int64_t nh = nb * kDigits;
    return (size_t)nh * sizeof(int64_t) + exclusive_scan_tmp_bytes(nh);
}

void radix_sort_u32(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt,
                    int64_t n, int bits, void *tmp, size_t tmp_bytes, bool *result_in_alt,
                    hipStream_t s) {
    radix_sort_impl<uint32_t>(keys, vals, keys_alt, vals_alt, n, bits, tmp, tmp_bytes,
                              result_in_alt, s);
}

void radix_sort_u64(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt,
                    int64_t n, int bits, void *tmp, size_t tmp_bytes, bool *result_in_alt,
                    hipStream_t s) {
    radix_sort_impl<uint64_t>(keys, vals, keys_alt, vals_alt, n, bits, tmp, tmp_bytes,
                              result_in_alt, s);
}

}  // namespace lowd
