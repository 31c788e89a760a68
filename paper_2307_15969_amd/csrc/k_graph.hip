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

// the same with each entry's value the edge's other end
__global__ void k_incidence_neighbours(int64_t m, const int32_t *src, const int32_t *dst,
                                       uint32_t *keys, uint32_t *vals) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < 2 * m;
         j += (int64_t)gridDim.x * blockDim.x) {
        const int64_t e = j >> 1;
        const uint32_t a = (uint32_t)src[e], b = (uint32_t)dst[e];
        keys[j] = (j & 1) ? b : a;
        vals[j] = (j & 1) ? a : b;
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

void build_incidence_ws(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, Arena &ws,
                        int64_t **row_ptr, uint32_t **inc, bool neighbours, hipStream_t s) {
    const int64_t len = 2 * m;
    const size_t cap = (size_t)(len > 0 ? len : 1);
    *row_ptr = ws.take<int64_t>((size_t)n + 1);
    *inc = ws.take<uint32_t>(cap);
    const size_t mk = ws.mark();
    uint32_t *k0 = ws.take<uint32_t>(cap), *k1 = ws.take<uint32_t>(cap);
    uint32_t *vt = ws.take<uint32_t>(cap);
    const size_t tmp_bytes = radix_sort_tmp_bytes(len);
    char *tmp = ws.take<char>(tmp_bytes);
    if (ws.base) {
        int bits = 1;
        while (bits < 32 && ((int64_t)1 << bits) < (int64_t)n) ++bits;
        // the sort makes one pass per 8 bits and ends in its second buffers
        // after an odd number of them: start the values where they end in inc
        const bool odd = len > 1 && ((bits + 7) / 8) % 2 == 1;
        uint32_t *v_in = odd ? vt : *inc, *v_alt = odd ? *inc : vt;
        if (len > 0) {
            if (neighbours)
                hipLaunchKernelGGL(k_incidence_neighbours, dim3(grid_for(len, 256)), dim3(256), 0,
                                   s, m, src, dst, k0, v_in);
            else
                hipLaunchKernelGGL(k_incidence_keys, dim3(grid_for(len, 256)), dim3(256), 0, s, m,
                                   src, dst, k0, v_in);
        }
        bool alt = false;
        radix_sort_u32(k0, v_in, k1, v_alt, len, bits, tmp, tmp_bytes, &alt, s);
        const uint32_t *keys = alt ? k1 : k0;
        hipLaunchKernelGGL(k_row_ptr, dim3(grid_for((int64_t)n + 1, 256)), dim3(256), 0, s, keys,
                           len, n, *row_ptr);
        if ((alt ? v_alt : v_in) != *inc && len > 0)
            LOWD_HIP(hipMemcpyAsync(*inc, alt ? v_alt : v_in, (size_t)len * sizeof(uint32_t),
                                    hipMemcpyDeviceToDevice, s));
        LOWD_HIP(hipGetLastError());
        LOWD_HIP(hipStreamSynchronize(s));
    }
    ws.release(mk);
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

}  // namespace

// Index of the later edge of the first repeated unordered pair found, or -1.
int64_t find_duplicate_pair_ws(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                               Arena &ws, hipStream_t s) {
    if (m < 2) return -1;
    const size_t mk = ws.mark();
    uint64_t *k0 = ws.take<uint64_t>((size_t)m), *k1 = ws.take<uint64_t>((size_t)m);
    uint32_t *v0 = ws.take<uint32_t>((size_t)m), *v1 = ws.take<uint32_t>((size_t)m);
    const size_t tmp_bytes = radix_sort_tmp_bytes(m);
    char *tmp = ws.take<char>(tmp_bytes);
    unsigned long long *bad = ws.take<unsigned long long>(1);
    unsigned int *any = ws.take<unsigned int>(1);
    unsigned long long r = ~0ull;
    if (ws.base) {
        int nb = 1;
        while (nb < 32 && ((int64_t)1 << nb) < (int64_t)n) ++nb;
        // Whether any pair repeats: the packed keys alone, sorted (2 nb bits).
        // Only then is the indexed sort below run, to name the edge.
        const unsigned int zero = 0u;
        LOWD_HIP(hipMemcpyAsync(any, &zero, sizeof(zero), hipMemcpyHostToDevice, s));
        hipLaunchKernelGGL(k_packed_pair_keys, dim3(grid_for(m, 256)), dim3(256), 0, s, m, src,
                           dst, nb, k0);
        bool alt = false;
        radix_sort_u64(k0, nullptr, k1, nullptr, m, 2 * nb, tmp, tmp_bytes, &alt, s);
        hipLaunchKernelGGL(k_any_adjacent_equal, dim3(grid_for(m, 256)), dim3(256), 0, s, m,
                           alt ? k1 : k0, any);
        LOWD_HIP(hipGetLastError());
        unsigned int found = 0u;
        LOWD_HIP(hipMemcpyAsync(&found, any, sizeof(found), hipMemcpyDeviceToHost, s));
        LOWD_HIP(hipStreamSynchronize(s));
        if (!found) {
            ws.release(mk);
            return -1;
        }
        hipLaunchKernelGGL(k_pair_keys, dim3(grid_for(m, 256)), dim3(256), 0, s, m, src, dst, k0,
                           v0);
        alt = false;
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
