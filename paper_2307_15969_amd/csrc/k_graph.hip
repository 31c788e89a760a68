// k_graph.hip -- input validation and the incidence CSR (node -> incident
// edge entries in ascending edge index), built with the stable radix sort.
#include <limits.h>

#include <utility>

#include "lowd_internal.h"

namespace lowd {
namespace {

__global__ void k_validate(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                           const float *w, unsigned long long *bad) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        int32_t a = src[e], b = dst[e];
        bool ok = a >= 0 && a < n && b >= 0 && b < n && a != b;
        if (w) {
            float x = w[e];
            ok = ok && (x > 0.0f) && (x <= 3.402823466e38f);   // positive and finite
        }
        if (!ok) atomicMin(bad, (unsigned long long)e);
    }
}

__global__ void k_incidence_keys(int64_t m, const int32_t *src, const int32_t *dst, uint32_t *keys,
                                 uint32_t *vals) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < 2 * m;
         j += (int64_t)gridDim.x * blockDim.x) {
        int64_t e = j >> 1;
        keys[j] = (uint32_t)((j & 1) ? dst[e] : src[e]);
        vals[j] = (uint32_t)j;
    }
}

// row_ptr[u] = first position of key u in the sorted keys (lower bound)
__global__ void k_row_ptr(const uint32_t *sorted, int64_t len, int32_t n, int64_t *row_ptr) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u <= n;
         u += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = len;
        while (lo < hi) {
            int64_t mid = (lo + hi) >> 1;
            if ((int64_t)sorted[mid] < u) lo = mid + 1;
            else hi = mid;
        }
        row_ptr[u] = lo;
    }
}

}  // namespace

void launch_validate(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, const float *w,
                     int64_t *bad_dev, hipStream_t s) {
    unsigned long long init = ULLONG_MAX;
    LOWD_HIP(hipMemcpyAsync(bad_dev, &init, sizeof(init), hipMemcpyHostToDevice, s));
    if (m > 0)
        hipLaunchKernelGGL(k_validate, dim3(grid_for(m, 256)), dim3(256), 0, s, n, m, src, dst, w,
                           (unsigned long long *)bad_dev);
    LOWD_HIP(hipGetLastError());
    LOWD_HIP(hipStreamSynchronize(s));   // `init` must outlive the copy
}

namespace {
// adj[j] = the other end of incidence entry j (entry = edge << 1 | side, side
// 1 when the row's node is the edge's dst)
__global__ void k_adjacency(int64_t len, const uint32_t *inc, const int32_t *src,
                            const int32_t *dst, int32_t *adj) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < len;
         j += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t ent = inc[j];
        adj[j] = (ent & 1u) ? src[ent >> 1] : dst[ent >> 1];
    }
}
}  // namespace

void build_adjacency(int64_t m, const Csr &csr, const int32_t *src, const int32_t *dst,
                     int32_t *adj, hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_adjacency, dim3(grid_for(2 * m, 256)), dim3(256), 0, s, 2 * m,
                       csr.inc.p, src, dst, adj);
    LOWD_HIP(hipGetLastError());
}

void build_incidence(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, Csr &csr,
                     hipStream_t s) {
    int64_t len = 2 * m;
    csr.row_ptr.alloc((size_t)n + 1);
    int bits = 1;
    while (bits < 32 && ((int64_t)1 << bits) < (int64_t)n) ++bits;
    size_t cap = (size_t)(len > 0 ? len : 1);
    DBuf<uint32_t> k0(cap), v0(cap), k1(cap), v1(cap);
    DBuf<char> tmp(radix_sort_tmp_bytes(len));
    if (len > 0)
        hipLaunchKernelGGL(k_incidence_keys, dim3(grid_for(len, 256)), dim3(256), 0, s, m, src, dst,
                           k0.p, v0.p);
    bool alt = false;
    radix_sort_u32(k0.p, v0.p, k1.p, v1.p, len, bits, tmp.p, tmp.bytes(), &alt, s);
    uint32_t *keys = alt ? k1.p : k0.p;
    hipLaunchKernelGGL(k_row_ptr, dim3(grid_for((int64_t)n + 1, 256)), dim3(256), 0, s, keys, len,
                       n, csr.row_ptr.p);
    LOWD_HIP(hipGetLastError());
    LOWD_HIP(hipStreamSynchronize(s));
    csr.inc = alt ? std::move(v1) : std::move(v0);
}

}  // namespace lowd

// --------------------------------------------------- repeated pairs ------
namespace lowd {
namespace {

__global__ void k_pair_keys(int64_t m, const int32_t *src, const int32_t *dst, uint64_t *keys,
                            uint32_t *vals) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        uint32_t a = (uint32_t)src[e], b = (uint32_t)dst[e];
        uint32_t lo = a < b ? a : b, hi = a < b ? b : a;
        keys[e] = ((uint64_t)lo << 32) | hi;
        vals[e] = (uint32_t)e;
    }
}

__global__ void k_adjacent_equal(int64_t m, const uint64_t *keys, const uint32_t *vals,
                                 unsigned long long *bad) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + 1; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        if (keys[i] == keys[i - 1]) atomicMin(bad, (unsigned long long)vals[i]);
}

// the unordered pair as one key of 2 nb bits: (smaller id << nb) | larger id
__global__ void k_packed_pair_keys(int64_t m, const int32_t *src, const int32_t *dst, int nb,
                                   uint64_t *keys) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t a = (uint32_t)src[e], b = (uint32_t)dst[e];
        keys[e] = a < b ? (a << nb) | b : (b << nb) | a;
    }
}

__global__ void k_any_adjacent_equal(int64_t m, const uint64_t *keys, unsigned int *any) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + 1; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        if (keys[i] == keys[i - 1]) *any = 1u;
}

// ---- repeated pairs by hash buckets ----
// The packed pair (2 nb <= 48 bits) goes to one of 2^bits buckets by a hash;
// the keys (pair << bits | bucket) sorted on their low `bits` bits put every
// bucket's pairs together (a repeated pair twice in one bucket), and one
// workgroup per bucket inserts them into a hash set in LDS.  A bucket too
// large for the set sends the check to the full sort instead.
constexpr int kRepeatBlock = 256;
constexpr int kRepeatCap = 5120;                 // pairs a bucket may hold
constexpr int kRepeatSlots = 2 * kRepeatCap;     // LDS set, half full at most
// 80 KB: two workgroups a CU
constexpr size_t kRepeatLds = (size_t)kRepeatSlots * sizeof(unsigned long long);
constexpr unsigned long long kRepeatEmpty = ~0ull;

// SplitMix64's output mix (Steele, Lea and Flood, OOPSLA 2014) as the hash
__device__ inline uint64_t pair_mix(uint64_t x) {
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// The bucketed keys; with `bad` the same pass also checks each edge as
// k_validate does (the keys of an invalid edge are never sorted: the check
// stops there).
__global__ void k_bucketed_pair_keys(int64_t m, const int32_t *src, const int32_t *dst, int nb,
                                     int bits, uint64_t *keys, int32_t n, const float *w,
                                     unsigned long long *bad) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t sa = src[e], sb = dst[e];
        if (bad) {
            bool ok = sa >= 0 && sa < n && sb >= 0 && sb < n && sa != sb;
            if (w) {
                const float x = w[e];
                ok = ok && (x > 0.0f) && (x <= 3.402823466e38f);   // positive and finite
            }
            if (!ok) atomicMin(bad, (unsigned long long)e);
        }
        const uint64_t a = (uint32_t)sa, b = (uint32_t)sb;
        const uint64_t pair = a < b ? (a << nb) | b : (b << nb) | a;
        keys[e] = (pair << bits) | (pair_mix(pair) >> (64 - bits));
    }
}

// start[b] = first position of bucket b in the keys sorted by bucket (b in
// [0, 2^bits]; start[2^bits] = m)
__global__ void k_bucket_starts(const uint64_t *keys, int64_t m, int bits, int64_t *start) {
    const int64_t nbk = (int64_t)1 << bits;
    const uint64_t mask = (uint64_t)nbk - 1;
    for (int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; b <= nbk;
         b += (int64_t)gridDim.x * blockDim.x) {
        int64_t lo = 0, hi = m;
        while (lo < hi) {
            const int64_t mid = (lo + hi) >> 1;
            if ((int64_t)(keys[mid] & mask) < b) lo = mid + 1;
            else hi = mid;
        }
        start[b] = lo;
    }
}

// flags[0] = 1 if a pair repeats, flags[1] = 1 if a bucket exceeded the set
__global__ void __launch_bounds__(kRepeatBlock)
    k_bucket_repeats(const uint64_t *keys, const int64_t *start, int bits, unsigned int *flags) {
    extern __shared__ unsigned long long set[];
    const int64_t nbk = (int64_t)1 << bits;
    for (int64_t b = blockIdx.x; b < nbk; b += gridDim.x) {   // uniform across the block
        const int64_t s0 = start[b], s1 = start[b + 1];
        if (s1 - s0 < 2) continue;
        if (s1 - s0 > kRepeatCap) {
            if (threadIdx.x == 0) flags[1] = 1u;
            continue;
        }
        for (int i = threadIdx.x; i < kRepeatSlots; i += kRepeatBlock) set[i] = kRepeatEmpty;
        __syncthreads();
        for (int64_t i = s0 + threadIdx.x; i < s1; i += kRepeatBlock) {
            const unsigned long long pair = keys[i] >> bits;
            // a slot from the low hash bits (the bucket took the top ones)
            uint32_t h = (uint32_t)(((uint64_t)(uint32_t)pair_mix(pair) * kRepeatSlots) >> 32);
            // the set is at most half full, so a free slot is always found
            for (;;) {
                const unsigned long long old = atomicCAS(&set[h], kRepeatEmpty, pair);
                if (old == kRepeatEmpty) break;
                if (old == pair) {
                    flags[0] = 1u;
                    break;
                }
                h = h + 1 == (uint32_t)kRepeatSlots ? 0u : h + 1;
            }
        }
        __syncthreads();
    }
}

}  // namespace

// Index of the later edge of the first repeated unordered pair found, or -1.
// Whether any pair repeats is decided first, by hash buckets (a radix sort
// of 8 to 24 bucket bits) or, where the ids are too wide for them or a
// bucket is too large, by a sort of the packed pairs; only when a pair
// repeats does an indexed sort of the pairs name the edge.  With `invalid`
// the edges are first checked as launch_validate does (in the pass that
// forms the bucketed keys, where the pairs are bucketed): *invalid receives
// the first invalid edge or -1, and the search for repeats runs only when
// there is none.
int64_t find_duplicate_pair_ws(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                               Arena &ws, hipStream_t s, const float *w, int64_t *invalid) {
    if (invalid) *invalid = -1;
    if (m < 2) {
        if (invalid && m > 0 && ws.base) {
            const size_t mk = ws.mark();
            int64_t *bad = ws.take<int64_t>(1);
            launch_validate(n, m, src, dst, w, bad, s);
            int64_t b = -1;
            LOWD_HIP(hipMemcpyAsync(&b, bad, sizeof(b), hipMemcpyDeviceToHost, s));
            LOWD_HIP(hipStreamSynchronize(s));
            if ((uint64_t)b != ~0ull) *invalid = b;
            ws.release(mk);
        } else if (invalid && m > 0) {
            (void)ws.take<int64_t>(1);
        }
        return -1;
    }
    int nb = 1;
    while (nb < 32 && ((int64_t)1 << nb) < (int64_t)n) ++nb;
    // bucket bits: buckets of at most about 2,048 pairs on average (well
    // within the set's capacity), at least 8 bits, at most 24 and what the
    // key leaves beside the pair
    int bits = 8;
    while (bits < 24 && ((int64_t)2048 << bits) < m) ++bits;
    bits = std::min(bits, 64 - 2 * nb);
    const bool bucketed = bits >= 8;
    const size_t mk = ws.mark();
    uint64_t *k0 = ws.take<uint64_t>((size_t)m), *k1 = ws.take<uint64_t>((size_t)m);
    uint32_t *v0 = ws.take<uint32_t>((size_t)m), *v1 = ws.take<uint32_t>((size_t)m);
    const size_t tmp_bytes = radix_sort_tmp_bytes(m);
    char *tmp = ws.take<char>(tmp_bytes);
    unsigned long long *bad = ws.take<unsigned long long>(1);
    unsigned int *flags = ws.take<unsigned int>(2);
    int64_t *bstart = bucketed ? ws.take<int64_t>(((size_t)1 << bits) + 1) : nullptr;
    unsigned long long r = ~0ull;
    if (ws.base) {
        const unsigned int zero[2] = {0u, 0u};
        unsigned int found[2] = {0u, 1u};
        if (bucketed) {
            static const bool lds_set = [] {
                LOWD_HIP(hipFuncSetAttribute((const void *)k_bucket_repeats,
                                             hipFuncAttributeMaxDynamicSharedMemorySize,
                                             (int)kRepeatLds));
                return true;
            }();
            (void)lds_set;
            LOWD_HIP(hipMemcpyAsync(flags, zero, sizeof(zero), hipMemcpyHostToDevice, s));
            const unsigned long long none = ~0ull;
            if (invalid)
                LOWD_HIP(hipMemcpyAsync(bad, &none, sizeof(none), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_bucketed_pair_keys, dim3(grid_for(m, 256)), dim3(256), 0, s, m,
                               src, dst, nb, bits, k0, n, w, invalid ? bad : nullptr);
            if (invalid) {
                unsigned long long b = ~0ull;
                LOWD_HIP(hipMemcpyAsync(&b, bad, sizeof(b), hipMemcpyDeviceToHost, s));
                LOWD_HIP(hipStreamSynchronize(s));
                if (b != ~0ull) {
                    *invalid = (int64_t)b;
                    ws.release(mk);
                    return -1;
                }
            }
            bool alt = false;
            radix_sort_u64(k0, nullptr, k1, nullptr, m, bits, tmp, tmp_bytes, &alt, s);
            const uint64_t *keys = alt ? k1 : k0;
            const int64_t nbk = (int64_t)1 << bits;
            hipLaunchKernelGGL(k_bucket_starts, dim3(grid_for(nbk + 1, 256)), dim3(256), 0, s,
                               keys, m, bits, bstart);
            hipLaunchKernelGGL(k_bucket_repeats, dim3(grid_for(nbk, 1, 8192)), dim3(kRepeatBlock),
                               kRepeatLds, s, keys, bstart, bits, flags);
            LOWD_HIP(hipGetLastError());
            LOWD_HIP(hipMemcpyAsync(found, flags, sizeof(found), hipMemcpyDeviceToHost, s));
            LOWD_HIP(hipStreamSynchronize(s));
        }
        if (!bucketed && invalid) {
            launch_validate(n, m, src, dst, w, (int64_t *)bad, s);
            unsigned long long b = ~0ull;
            LOWD_HIP(hipMemcpyAsync(&b, bad, sizeof(b), hipMemcpyDeviceToHost, s));
            LOWD_HIP(hipStreamSynchronize(s));
            if (b != ~0ull) {
                *invalid = (int64_t)b;
                ws.release(mk);
                return -1;
            }
        }
        if (found[1]) {
            // the packed keys alone, sorted (2 nb bits)
            LOWD_HIP(hipMemcpyAsync(flags, zero, sizeof(zero), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_packed_pair_keys, dim3(grid_for(m, 256)), dim3(256), 0, s, m,
                               src, dst, nb, k0);
            bool alt = false;
            radix_sort_u64(k0, nullptr, k1, nullptr, m, 2 * nb, tmp, tmp_bytes, &alt, s);
            hipLaunchKernelGGL(k_any_adjacent_equal, dim3(grid_for(m, 256)), dim3(256), 0, s, m,
                               alt ? k1 : k0, flags);
            LOWD_HIP(hipGetLastError());
            LOWD_HIP(hipMemcpyAsync(found, flags, sizeof(unsigned int), hipMemcpyDeviceToHost,
                                    s));
            LOWD_HIP(hipStreamSynchronize(s));
        }
        if (!found[0]) {
            ws.release(mk);
            return -1;
        }
        hipLaunchKernelGGL(k_pair_keys, dim3(grid_for(m, 256)), dim3(256), 0, s, m, src, dst, k0,
                           v0);
        bool alt = false;
        radix_sort_u64(k0, v0, k1, v1, m, 32 + nb, tmp, tmp_bytes, &alt, s);
        unsigned long long init = ~0ull;
        LOWD_HIP(hipMemcpyAsync(bad, &init, sizeof(init), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_adjacent_equal, dim3(grid_for(m, 256)), dim3(256), 0, s, m,
                           alt ? k1 : k0, alt ? v1 : v0, bad);
        LOWD_HIP(hipGetLastError());
        LOWD_HIP(hipMemcpyAsync(&r, bad, sizeof(r), hipMemcpyDeviceToHost, s));
        LOWD_HIP(hipStreamSynchronize(s));
    }
    ws.release(mk);
    return r == ~0ull ? -1 : (int64_t)r;
}

int64_t find_duplicate_pair(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                            hipStream_t s) {
    if (m < 2) return -1;
    Arena measure;
    find_duplicate_pair_ws(n, m, src, dst, measure, s);
    DBuf<char> buf(measure.peak);
    Arena ws(buf.p, buf.bytes());
    return find_duplicate_pair_ws(n, m, src, dst, ws, s);
}

}  // namespace lowd
