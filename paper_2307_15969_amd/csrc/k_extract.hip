// k_extract.hip -- Algorithm 1's extraction on the GPU: a stable ascending
// sort of the FP64 loads (ties by node id), the weight W(S_i) of every
// remaining set S_i = V minus the first i sorted nodes, and the first index
// of maximal density W(S_i) / (n - i).
//
// An edge lies inside S_i exactly when both endpoints sit at position >= i,
// so W(S_i) is the suffix sum of the weights binned at min(pos_u, pos_v).
// Unweighted graphs bin with integer atomics and use int64 throughout, so
// densities compare exactly by cross-multiplication; weighted graphs sum
// each node's weight towards higher positions over its incidence row.
#include "extract.h"
#include "lowd_internal.h"

namespace lowd {
namespace {

// order-preserving map of an FP64 value onto uint64 (-0 folded onto +0)
__device__ inline uint64_t sortable(double v) {
    v = v + 0.0;
    uint64_t b = __builtin_bit_cast(uint64_t, v);
    return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}

__global__ void k_keys(int32_t n, const double *L, uint64_t *keys, uint32_t *vals) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x) {
        keys[u] = sortable(L[u]);
        vals[u] = (uint32_t)u;
    }
}

__global__ void k_positions(int32_t n, const uint32_t *asc, int32_t *pos) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        pos[asc[i]] = (int32_t)i;
}

// Unweighted: each edge adds 1 at min(pos_u, pos_v) (integer atomics, exact
// in any order).
__global__ void k_fill_i64(int64_t n, int64_t *a) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = 0;
}

__global__ void k_edge_min_pos(int64_t m, const int32_t *src, const int32_t *dst,
                               const int32_t *pos, unsigned long long *hist) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        int32_t a = pos[src[e]], b = pos[dst[e]];
        atomicAdd(&hist[a < b ? a : b], 1ull);
    }
}

// Unweighted, without atomics: node u's bin is the number of its neighbours
// at higher positions (positions are distinct, so every edge is counted once,
// at its lower end).  Groups of 8 lanes per node of degree below kBigRow;
// the others are left to k_towards_higher_big.  Writes every such bin.
constexpr int kRowLanes = 8;
__global__ void __launch_bounds__(256) k_towards_higher_small(int32_t n, const int64_t *row_ptr,
                                                              const int32_t *adj,
                                                              const int32_t *pos,
                                                              unsigned long long *hist) {
    const int sub = threadIdx.x & (kRowLanes - 1);
    const int64_t groups = (int64_t)gridDim.x * (blockDim.x / kRowLanes);
    for (int64_t u = (int64_t)blockIdx.x * (blockDim.x / kRowLanes) + threadIdx.x / kRowLanes;
         u < n; u += groups) {
        const int64_t b = row_ptr[u], e = row_ptr[u + 1];
        if (e - b >= kBigRow) continue;   // the whole group skips it
        const int32_t pu = pos[u];
        uint32_t c = 0;
        for (int64_t j = b + sub; j < e; j += kRowLanes) c += pos[adj[j]] > pu ? 1u : 0u;
        for (int d = kRowLanes / 2; d > 0; d >>= 1) c += __shfl_down(c, d, kRowLanes);
        if (sub == 0) hist[pu] = c;
    }
}

// One workgroup per node of degree >= kBigRow (the list big[]).
constexpr int kBigBlock = 256;
__global__ void __launch_bounds__(kBigBlock) k_towards_higher_big(const int32_t *big,
                                                                  const int64_t *row_ptr,
                                                                  const int32_t *adj,
                                                                  const int32_t *pos,
                                                                  unsigned long long *hist) {
    __shared__ uint32_t part[kBigBlock / kWave];
    const int32_t u = big[blockIdx.x];
    const int32_t pu = pos[u];
    uint32_t c = 0;
    for (int64_t j = row_ptr[u] + threadIdx.x; j < row_ptr[u + 1]; j += kBigBlock)
        c += pos[adj[j]] > pu ? 1u : 0u;
    for (int d = kWave / 2; d > 0; d >>= 1) c += __shfl_down(c, d, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int k = 0; k < kBigBlock / kWave; ++k) t += part[k];
        hist[pu] = t;
    }
}

// Weighted: the weight from node u towards nodes at higher positions, stored
// at pos[u], summed exactly: each weight is the integer wi[e] (the weight
// over 2^q, see fixed_point_weights), so the sums are exact 128-bit integers
// in any order.  The weights are read per incidence entry (wi_inc, in row
// order) rather than gathered by edge.  Groups of 8 lanes per node of
// degree below kBigRow (the others: k_towards_higher_w_big).
__device__ __forceinline__ u128 shfl_down_u128(u128 v, int d, int width) {
    struct Words {
        int w[4];
    };
    Words x = __builtin_bit_cast(Words, v);
#pragma unroll
    for (int k = 0; k < 4; ++k) x.w[k] = __shfl_down(x.w[k], d, width);
    return __builtin_bit_cast(u128, x);
}

__global__ void __launch_bounds__(256) k_towards_higher_w(int32_t n, const int64_t *row_ptr,
                                                          const int32_t *adj,
                                                          const uint64_t *wi_inc,
                                                          const int32_t *pos, u128 *hist) {
    const int sub = threadIdx.x & (kRowLanes - 1);
    const int64_t groups = (int64_t)gridDim.x * (blockDim.x / kRowLanes);
    for (int64_t u = (int64_t)blockIdx.x * (blockDim.x / kRowLanes) + threadIdx.x / kRowLanes;
         u < n; u += groups) {
        const int64_t b = row_ptr[u], e = row_ptr[u + 1];
        if (e - b >= kBigRow) continue;
        const int32_t pu = pos[u];
        u128 acc = 0;
        for (int64_t j = b + sub; j < e; j += kRowLanes)
            if (pos[adj[j]] > pu) acc += (u128)wi_inc[j];
        for (int d = kRowLanes / 2; d > 0; d >>= 1) acc += shfl_down_u128(acc, d, kRowLanes);
        if (sub == 0) hist[pu] = acc;
    }
}

// the same for one node of degree >= kBigRow per workgroup
__global__ void __launch_bounds__(kBigBlock) k_towards_higher_w_big(
    const int32_t *big, const int64_t *row_ptr, const int32_t *adj, const uint64_t *wi_inc,
    const int32_t *pos, u128 *hist) {
    __shared__ u128 part[kBigBlock / kWave];
    const int32_t u = big[blockIdx.x];
    const int32_t pu = pos[u];
    u128 acc = 0;
    for (int64_t j = row_ptr[u] + threadIdx.x; j < row_ptr[u + 1]; j += kBigBlock)
        if (pos[adj[j]] > pu) acc += (u128)wi_inc[j];
    for (int d = kWave / 2; d > 0; d >>= 1) acc += shfl_down_u128(acc, d, kWave);
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        u128 t = 0;
        for (int k = 0; k < kBigBlock / kWave; ++k) t += part[k];
        hist[pu] = t;
    }
}

// W(S_i) from the exclusive prefix P of the reversed histogram:
// W[i] = P[n-1-i] + hist[i]
template <class T>
__global__ void k_reverse(int64_t n, const T *in, T *out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[n - 1 - i] = in[i];
}

template <class T>
__global__ void k_suffix(int64_t n, const T *prefix_rev, const T *hist, T *W) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        W[i] = prefix_rev[n - 1 - i] + hist[i];
}

// is candidate i strictly better than j (denser, or as dense and larger)?
__device__ inline bool better(int64_t i, int64_t j, const int64_t *W, int64_t n) {
    if (j < 0) return i >= 0;
    if (i < 0) return false;
    // W_i / (n-i) vs W_j / (n-j), exact in int64 (W < 2^31, n < 2^31)
    int64_t a = W[i] * (n - j), b = W[j] * (n - i);
    return a > b || (a == b && i < j);
}
// weighted, exact: W < 2^95 (integer weights below 2^64, fewer than 2^31
// edges) and n < 2^31, so the cross products stay below 2^126
__device__ inline bool better(int64_t i, int64_t j, const u128 *W, int64_t n) {
    if (j < 0) return i >= 0;
    if (i < 0) return false;
    const u128 a = W[i] * (u128)(n - j), b = W[j] * (u128)(n - i);
    return a > b || (a == b && i < j);
}

constexpr int kArgBlock = 256;

template <class T>
__device__ inline int64_t block_best(int64_t cand, const T *W, int64_t n, int64_t *lds) {
    lds[threadIdx.x] = cand;
    __syncthreads();
    for (int s = kArgBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            int64_t o = lds[threadIdx.x + s];
            if (better(o, lds[threadIdx.x], W, n)) lds[threadIdx.x] = o;
        }
        __syncthreads();
    }
    return lds[0];
}

template <class T>
__global__ void __launch_bounds__(kArgBlock) k_best_partial(int64_t n, const T *W, int64_t *part) {
    __shared__ int64_t lds[kArgBlock];
    int64_t cand = -1;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        if (better(i, cand, W, n)) cand = i;
    int64_t b = block_best(cand, W, n, lds);
    if (threadIdx.x == 0) part[blockIdx.x] = b;
}

template <class T>
__global__ void __launch_bounds__(kArgBlock) k_best_final(int64_t n, int32_t nb, const int64_t *part,
                                                          const T *W, int64_t *best, T *best_w) {
    __shared__ int64_t lds[kArgBlock];
    int64_t cand = -1;
    for (int32_t b = threadIdx.x; b < nb; b += blockDim.x)
        if (better(part[b], cand, W, n)) cand = part[b];
    int64_t r = block_best(cand, W, n, lds);
    if (threadIdx.x == 0) {
        *best = r;
        *best_w = W[r];
    }
}

__global__ void k_in_set(int32_t n, const int32_t *pos, const int64_t *best, uint8_t *in_set) {
    const int64_t b = *best;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x)
        in_set[u] = pos[u] >= b ? 1 : 0;
}

template <class T, bool kWeighted>
void extract_impl(const ExtractArgs &a, ExtractScratch &sc, hipStream_t s) {
    const int32_t n = a.n;
    hipLaunchKernelGGL(k_keys, dim3(grid_for(n, 256)), dim3(256), 0, s, n, a.L64, sc.keys.p,
                       sc.vals.p);
    bool alt = false;
    radix_sort_u64(sc.keys.p, sc.vals.p, sc.keys_alt.p, sc.vals_alt.p, n, 64, sc.tmp.p,
                   sc.tmp.bytes(), &alt, s);
    const uint32_t *asc = alt ? sc.vals_alt.p : sc.vals.p;
    hipLaunchKernelGGL(k_positions, dim3(grid_for(n, 256)), dim3(256), 0, s, n, asc, sc.pos.p);
    T *hist = (T *)sc.hist.p;
    T *rev = (T *)sc.rev.p;
    T *W = (T *)sc.W.p;
    if constexpr (kWeighted) {
        if (a.m == 0) {   // no edges: every bin is zero
            hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(2 * (int64_t)n, 256)), dim3(256), 0, s,
                               2 * (int64_t)n, (int64_t *)hist);
        } else {
            if (!a.adj || !a.wi_inc)
                fail(LOWD_E_ARG, "weighted extraction needs the adjacency and entry weights");
            hipLaunchKernelGGL(k_towards_higher_w, dim3(grid_for((int64_t)n * kRowLanes, 256)),
                               dim3(256), 0, s, n, a.row_ptr, a.adj, a.wi_inc, sc.pos.p, hist);
        }
        if (a.m > 0 && a.nbig > 0)
            hipLaunchKernelGGL(k_towards_higher_w_big, dim3((unsigned)a.nbig), dim3(kBigBlock), 0,
                               s, a.big, a.row_ptr, a.adj, a.wi_inc, sc.pos.p, hist);
    } else if (a.adj) {
        hipLaunchKernelGGL(k_towards_higher_small, dim3(grid_for((int64_t)n * kRowLanes, 256)),
                           dim3(256), 0, s, n, a.row_ptr, a.adj, sc.pos.p,
                           (unsigned long long *)hist);
        if (a.nbig > 0)
            hipLaunchKernelGGL(k_towards_higher_big, dim3((unsigned)a.nbig), dim3(kBigBlock), 0, s,
                               a.big, a.row_ptr, a.adj, sc.pos.p, (unsigned long long *)hist);
    } else {
        hipLaunchKernelGGL(k_fill_i64, dim3(grid_for(n, 256)), dim3(256), 0, s, (int64_t)n, hist);
        if (a.m > 0)
            hipLaunchKernelGGL(k_edge_min_pos, dim3(grid_for(a.m, 256)), dim3(256), 0, s, a.m,
                               a.src, a.dst, sc.pos.p, (unsigned long long *)hist);
    }
    hipLaunchKernelGGL(k_reverse<T>, dim3(grid_for(n, 256)), dim3(256), 0, s, (int64_t)n, hist,
                       rev);
    if constexpr (kWeighted)
        exclusive_scan_u128(rev, rev, n, nullptr, sc.tmp.p, sc.tmp.bytes(), s);
    else
        exclusive_scan_i64(rev, rev, n, nullptr, sc.tmp.p, sc.tmp.bytes(), s);
    hipLaunchKernelGGL(k_suffix<T>, dim3(grid_for(n, 256)), dim3(256), 0, s, (int64_t)n, rev, hist,
                       W);
    int32_t nb = (int32_t)grid_for(n, kArgBlock, 1024);
    hipLaunchKernelGGL(k_best_partial<T>, dim3((unsigned)nb), dim3(kArgBlock), 0, s, (int64_t)n, W,
                       sc.part.p);
    hipLaunchKernelGGL(k_best_final<T>, dim3(1), dim3(kArgBlock), 0, s, (int64_t)n, nb, sc.part.p,
                       W, sc.best.p, (T *)(sc.best.p + 1));
    hipLaunchKernelGGL(k_in_set, dim3(grid_for(n, 256)), dim3(256), 0, s, n, sc.pos.p, sc.best.p,
                       a.in_set);
    LOWD_HIP(hipGetLastError());
}

}  // namespace

void ExtractScratch::ensure(int64_t n) {
    if (cap >= n) return;
    int64_t c = n > 0 ? n : 1;
    keys.alloc((size_t)c);
    keys_alt.alloc((size_t)c);
    vals.alloc((size_t)c);
    vals_alt.alloc((size_t)c);
    pos.alloc((size_t)c);
    hist.alloc(2 * (size_t)c);   // room for 128-bit weighted sums
    rev.alloc(2 * (size_t)c);
    W.alloc(2 * (size_t)c);
    part.alloc(1024);
    best.alloc(3);
    size_t t = radix_sort_tmp_bytes(c);
    size_t t2 = exclusive_scan_tmp_bytes(c);
    tmp.alloc(t > t2 ? t : t2);
    cap = c;
}

void launch_extract(const ExtractArgs &a, ExtractScratch &sc, hipStream_t s) {
    sc.ensure(a.n);
    if (a.weighted) extract_impl<u128, true>(a, sc, s);
    else extract_impl<int64_t, false>(a, sc, s);
}

}  // namespace lowd

// ------------------------------------------------ decomposition read-out --
// The locally-dense decomposition read from the loads (Problem 2, Property
// 2): with the nodes ranked by descending load (the reverse of the
// extraction's order) and f(k) the weight induced by the top k nodes
// (f(k) = W(S_{n-k}), f(0) = 0), each level ends at the largest k that
// maximises the average (f(k) - f(k_prev)) / (k - k_prev) beyond the
// previous level.  Those ends are the strict corners of the upper concave
// hull of the points (k, f(k)), k = 0..n.  The hull is built in two steps:
// every chunk of 256 points reduces to its own hull vertices (one thread
// per chunk, a monotone chain), and one thread chains the surviving
// candidates in order (a vertex of the whole hull is a vertex of its chunk's
// hull).  Unit weights decide every turn exactly in 128-bit integers.
namespace lowd {
namespace {

constexpr int64_t kHullChunk = 256;

template <class T>
__device__ __forceinline__ T f_at(const T *W, int64_t n, int64_t k) {
    return k == 0 ? (T)0 : W[n - k];
}

// is a not strictly above the segment from o to b?  (cross product >= 0)
__device__ __forceinline__ bool not_above(int64_t ok, int64_t of, int64_t ak, int64_t af,
                                          int64_t bk, int64_t bf) {
    const __int128 l = (__int128)(ak - ok) * (__int128)(bf - of);
    const __int128 r = (__int128)(af - of) * (__int128)(bk - ok);
    return l >= r;
}
// weighted, exact: f is non-decreasing in k, so the differences are
// non-negative; f < 2^95 and k < 2^31 keep the products below 2^126
__device__ __forceinline__ bool not_above(int64_t ok, u128 of, int64_t ak, u128 af, int64_t bk,
                                          u128 bf) {
    const u128 l = (u128)(ak - ok) * (bf - of);
    const u128 r = (af - of) * (u128)(bk - ok);
    return l >= r;
}

// f(k) as FP64: exact integers for unit weights; the weighted integer sum
// (in units of 2^q) rounded once and scaled
__device__ __forceinline__ double f_value(int64_t v, int32_t) { return (double)v; }
__device__ __forceinline__ double f_value(u128 v, int32_t q) { return ldexp(u128_to_double(v), q); }

template <class T>
__global__ void k_hull_chunks(int64_t n, const T *W, int64_t *ck, T *cf, int64_t *cnt) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t lo = c * kHullChunk;
    if (lo > n) return;
    const int64_t hi = lo + kHullChunk < n + 1 ? lo + kHullChunk : n + 1;
    int64_t *sk = ck + lo;
    T *sf = cf + lo;
    int64_t top = 0;
    for (int64_t k = lo; k < hi; ++k) {
        const T f = f_at(W, n, k);
        while (top >= 2 && not_above(sk[top - 2], sf[top - 2], sk[top - 1], sf[top - 1], k, f))
            --top;
        sk[top] = k;
        sf[top] = f;
        ++top;
    }
    cnt[c] = top;
}

template <class T>
__global__ void k_hull_compact(int64_t chunks, const int64_t *ck, const T *cf, const int64_t *cnt,
                               const int64_t *off, int64_t *qk, T *qf) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= chunks) return;
    const int64_t lo = c * kHullChunk;
    for (int64_t i = 0; i < cnt[c]; ++i) {
        qk[off[c] + i] = ck[lo + i];
        qf[off[c] + i] = cf[lo + i];
    }
}

// one thread: the monotone chain over the candidates; hk/hf receive the hull
// vertices k_0 = 0 < k_1 < ... < k_L = n and *nv = L + 1
template <class T>
__global__ void k_hull_chain(int64_t q, const int64_t *qk, const T *qf, int64_t *hk, T *hf,
                             int64_t *nv) {
    if (blockIdx.x != 0 || threadIdx.x != 0) return;
    int64_t top = 0;
    for (int64_t i = 0; i < q; ++i) {
        const int64_t k = qk[i];
        const T f = qf[i];
        while (top >= 2 && not_above(hk[top - 2], hf[top - 2], hk[top - 1], hf[top - 1], k, f))
            --top;
        hk[top] = k;
        hf[top] = f;
        ++top;
    }
    *nv = top;
}

// level of every node: the number of level ends k_j (j >= 1) at or below its
// descending rank; and the ends as output arrays
template <class T>
__global__ void k_hull_levels(int32_t n, const int32_t *pos, const int64_t *hk, const T *hf,
                              const int64_t *nv, int32_t q, int32_t *level, int64_t *k_end,
                              double *f_end) {
    const int64_t L = *nv - 1;
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = (int64_t)n - 1 - pos[u];
        int64_t a = 1, b = L + 1;   // first j in [1, L] with hk[j] > r
        while (a < b) {
            const int64_t mid = (a + b) >> 1;
            if (hk[mid] <= r) a = mid + 1;
            else b = mid;
        }
        level[u] = (int32_t)(a - 1);
        if (u < L) {
            k_end[u] = hk[u + 1];
            f_end[u] = f_value(hf[u + 1], q);
        }
    }
}

template <class T>
void ldd_impl(int32_t n, int32_t q, const ExtractScratch &sc, LddScratch &ls, int32_t *level,
              int64_t *k_end, double *f_end, hipStream_t s) {
    const T *W = (const T *)sc.W.p;
    const int64_t pts = (int64_t)n + 1;
    const int64_t chunks = (pts + kHullChunk - 1) / kHullChunk;
    ls.ensure(pts, chunks);
    int64_t *ck = ls.ck.p, *qk = ls.qk.p, *hk = ls.hk.p;
    T *cf = (T *)ls.cf.p, *qf = (T *)ls.qf.p, *hf = (T *)ls.hf.p;
    hipLaunchKernelGGL(k_hull_chunks<T>, dim3(grid_for(chunks, 64)), dim3(64), 0, s, (int64_t)n, W,
                       ck, cf, ls.cnt.p);
    int64_t *total = ls.cnt.p + chunks;   // the scan's total, one past the counts
    exclusive_scan_i64(ls.cnt.p, ls.off.p, chunks, total, ls.tmp.p, ls.tmp.bytes(), s);
    hipLaunchKernelGGL(k_hull_compact<T>, dim3(grid_for(chunks, 64)), dim3(64), 0, s, chunks, ck,
                       cf, ls.cnt.p, ls.off.p, qk, qf);
    LOWD_HIP(hipMemcpyAsync(&ls.host_q, total, sizeof(int64_t), hipMemcpyDeviceToHost, s));
    LOWD_HIP(hipStreamSynchronize(s));
    hipLaunchKernelGGL(k_hull_chain<T>, dim3(1), dim3(64), 0, s, ls.host_q, qk, qf, hk, hf,
                       ls.nv.p);
    hipLaunchKernelGGL(k_hull_levels<T>, dim3(grid_for(n, 256)), dim3(256), 0, s, n, sc.pos.p, hk,
                       hf, ls.nv.p, q, level, k_end, f_end);
    LOWD_HIP(hipGetLastError());
}

}  // namespace

void LddScratch::ensure(int64_t points, int64_t chunks) {
    if (points <= cap_points && chunks <= cap_chunks) return;
    ck.alloc((size_t)points);
    cf.alloc(2 * (size_t)points);   // room for 128-bit weighted values
    qk.alloc((size_t)points);
    qf.alloc(2 * (size_t)points);
    hk.alloc((size_t)points);
    hf.alloc(2 * (size_t)points);
    cnt.alloc((size_t)chunks + 1);
    off.alloc((size_t)chunks);
    nv.alloc(1);
    tmp.alloc(exclusive_scan_tmp_bytes(chunks));
    cap_points = points;
    cap_chunks = chunks;
}

void launch_ldd(const ExtractArgs &a, ExtractScratch &sc, LddScratch &ls, int32_t *level,
                int64_t *k_end, double *f_end, int64_t *nlevels, hipStream_t s) {
    launch_extract(a, sc, s);   // order, positions and W(S_i)
    if (a.weighted) ldd_impl<u128>(a.n, a.wq, sc, ls, level, k_end, f_end, s);
    else ldd_impl<int64_t>(a.n, 0, sc, ls, level, k_end, f_end, s);
    int64_t nv = 0;
    LOWD_HIP(hipMemcpyAsync(&nv, ls.nv.p, sizeof(nv), hipMemcpyDeviceToHost, s));
    LOWD_HIP(hipStreamSynchronize(s));
    *nlevels = nv - 1;
}

}  // namespace lowd

// ------------------------------------------------ batched extraction -----
// The same extraction for many graphs at once (unweighted), over the graphs
// still iterating: act[k] (k < A) is the k-th of them, and its nodes take
// the compact range seg[k] .. seg[k+1]-1.  One stable sort of their loads,
// then a stable sort by k, gives every graph's ascending order as its
// compact range; positions, the W(S_i) suffix sums and the densest prefix
// are then taken per range.
namespace lowd {
namespace {

// one block per listed graph: its nodes' sort keys and ids, in compact order
__global__ void k_keys_batch(int32_t A, const int32_t *act, const int64_t *seg,
                             const int64_t *node_ptr, const double *L, uint64_t *keys,
                             uint32_t *vals) {
    for (int32_t k = blockIdx.x; k < A; k += gridDim.x) {
        const int32_t g = act[k];
        const int64_t u0 = node_ptr[g], c0 = seg[k];
        const int64_t n = node_ptr[g + 1] - u0;
        for (int64_t j = threadIdx.x; j < n; j += blockDim.x) {
            keys[c0 + j] = sortable(L[u0 + j]);
            vals[c0 + j] = (uint32_t)(u0 + j);
        }
    }
}

__global__ void k_graph_keys(int64_t Na, const uint32_t *vals, const int32_t *node_graph,
                             const int32_t *rank, uint32_t *keys2) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < Na;
         k += (int64_t)gridDim.x * blockDim.x)
        keys2[k] = (uint32_t)rank[node_graph[vals[k]]];
}

// Compact positions in the sorted order, which keeps each graph's nodes
// together (the k-th listed graph at seg[k] .. seg[k+1]-1): node u's
// position within its graph is pos[u] - seg[k].
__global__ void k_batch_positions(int64_t Na, const uint32_t *asc, int32_t *pos) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < Na;
         k += (int64_t)gridDim.x * blockDim.x)
        pos[asc[k]] = (int32_t)k;
}

// Both ends of an edge are in one graph, so the smaller compact position is
// the graph's offset plus the smaller position within the graph.  Edges of
// graphs not listed are skipped.
__global__ void k_edge_min_pos_batch(int64_t M, const int32_t *gsrc, const int32_t *gdst,
                                     const int32_t *node_graph, const int32_t *rank,
                                     const int32_t *pos, unsigned long long *hist) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < M;
         e += (int64_t)gridDim.x * blockDim.x) {
        if (rank[node_graph[gsrc[e]]] < 0) continue;
        const int32_t a = pos[gsrc[e]], b = pos[gdst[e]];
        atomicAdd(&hist[a < b ? a : b], 1ull);
    }
}

// one block per listed graph: first index of maximal density W_g[i] / (n_g - i),
// and the graph's largest load D_g (the dual bound of Section III-B)
__global__ void __launch_bounds__(kArgBlock) k_best_batch(int32_t A, const int32_t *act,
                                                          const int64_t *seg,
                                                          const int64_t *node_ptr, int64_t Na,
                                                          const int64_t *W, const double *L64,
                                                          int64_t *best, int64_t *num,
                                                          int64_t *den, double *D) {
    __shared__ int64_t lds_i[kArgBlock];
    __shared__ int64_t lds_w[kArgBlock];
    __shared__ double lds_d[kArgBlock];
    const int32_t k = blockIdx.x;
    const int32_t g = act[k];
    const int64_t start = seg[k], end = seg[k + 1];
    const int64_t n = end - start, u0 = node_ptr[g];
    const int64_t tail = end < Na ? W[end] : 0;
    int64_t bi = -1, bw = 0;
    double dmax = -1.0e308;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        const int64_t wi = W[start + i] - tail;
        // wi / (n - i) > bw / (n - bi), exact in int64
        if (bi < 0 || wi * (n - bi) > bw * (n - i)) { bi = i; bw = wi; }
        const double l = L64[u0 + i];
        dmax = l > dmax ? l : dmax;
    }
    lds_i[threadIdx.x] = bi;
    lds_w[threadIdx.x] = bw;
    lds_d[threadIdx.x] = dmax;
    __syncthreads();
    for (int s = kArgBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            const double od = lds_d[threadIdx.x + s];
            if (od > lds_d[threadIdx.x]) lds_d[threadIdx.x] = od;
            const int64_t oi = lds_i[threadIdx.x + s], ow = lds_w[threadIdx.x + s];
            const int64_t ci = lds_i[threadIdx.x], cw = lds_w[threadIdx.x];
            bool take;
            if (oi < 0) take = false;
            else if (ci < 0) take = true;
            else {
                const int64_t a = ow * (n - ci), b = cw * (n - oi);
                take = a > b || (a == b && oi < ci);
            }
            if (take) { lds_i[threadIdx.x] = oi; lds_w[threadIdx.x] = ow; }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        best[k] = lds_i[0];
        num[g] = lds_w[0];
        den[g] = n - lds_i[0];
        D[g] = lds_d[0];
    }
}

// One workgroup per listed graph: each edge's smaller position is counted in
// LDS (a graph's nodes fit one workgroup's LDS), then the graph's bins are
// written out.  Counts are integers, so the order of the additions does not
// matter.  Writes every bin of hist[0 .. seg[A]).
constexpr int kGraphHistBlock = 256;
constexpr size_t kGraphHistLds = 160 * 1024;   // a CU's LDS
__global__ void __launch_bounds__(kGraphHistBlock)
k_edge_min_pos_graph(const int32_t *act, const int64_t *seg, const int64_t *edge_ptr,
                     const int32_t *gsrc, const int32_t *gdst, const int32_t *pos,
                     unsigned long long *hist) {
    extern __shared__ uint32_t hbin[];
    const int32_t k = (int32_t)blockIdx.x;
    const int32_t g = act[k];
    const int64_t base = seg[k];
    const int32_t n = (int32_t)(seg[k + 1] - base);
    for (int32_t i = threadIdx.x; i < n; i += kGraphHistBlock) hbin[i] = 0u;
    __syncthreads();
    const int64_t e1 = edge_ptr[g + 1];
    for (int64_t e = edge_ptr[g] + threadIdx.x; e < e1; e += kGraphHistBlock) {
        const int32_t a = pos[gsrc[e]], b = pos[gdst[e]];
        atomicAdd(&hbin[(a < b ? a : b) - base], 1u);
    }
    __syncthreads();
    for (int32_t i = threadIdx.x; i < n; i += kGraphHistBlock) hist[base + i] = hbin[i];
}

// one block per listed graph: its nodes' membership in its densest prefix
__global__ void k_in_set_batch(int32_t A, const int32_t *act, const int64_t *seg,
                               const int64_t *node_ptr, const int32_t *pos, const int64_t *best,
                               uint8_t *in_set) {
    for (int32_t k = blockIdx.x; k < A; k += gridDim.x) {
        const int32_t g = act[k];
        const int64_t u0 = node_ptr[g], n = node_ptr[g + 1] - u0, c0 = seg[k], bk = best[k];
        for (int64_t j = threadIdx.x; j < n; j += blockDim.x)
            in_set[u0 + j] = (int64_t)pos[u0 + j] - c0 >= bk ? 1 : 0;
    }
}

}  // namespace

void BatchExtractScratch::ensure(int64_t N, int32_t G) {
    if (N <= cap_n && G <= cap_g) return;
    const size_t n = (size_t)(N > 0 ? N : 1);
    k0.alloc(n);
    k1.alloc(n);
    v0.alloc(n);
    v1.alloc(n);
    g0.alloc(n);
    g1.alloc(n);
    pos.alloc(n);
    hist.alloc(n);
    rev.alloc(n);
    W.alloc(n);
    best.alloc((size_t)(G > 0 ? G : 1));
    const size_t tb = radix_sort_tmp_bytes(N), tb2 = exclusive_scan_tmp_bytes(N);
    tmp.alloc(tb > tb2 ? tb : tb2);
    cap_n = N;
    cap_g = G;
}

void launch_extract_batch(const BatchExtractArgs &a, BatchExtractScratch &sc, hipStream_t s) {
    const int64_t Na = a.Na;
    if (a.A <= 0 || Na <= 0) return;
    int gbits = 1;
    while (gbits < 31 && ((int64_t)1 << gbits) < (int64_t)a.A) ++gbits;
    sc.ensure(a.N, a.G);
    const unsigned gn = grid_for(Na, 256);
    const unsigned ga = (unsigned)(a.A < 65535 ? a.A : 65535);
    hipLaunchKernelGGL(k_keys_batch, dim3(ga), dim3(256), 0, s, a.A, a.act, a.seg, a.node_ptr,
                       a.L64, sc.k0.p, sc.v0.p);
    bool alt = false;
    radix_sort_u64(sc.k0.p, sc.v0.p, sc.k1.p, sc.v1.p, Na, 64, sc.tmp.p, sc.tmp.bytes(), &alt, s);
    uint32_t *vals = alt ? sc.v1.p : sc.v0.p;
    uint32_t *vals_alt = alt ? sc.v0.p : sc.v1.p;
    hipLaunchKernelGGL(k_graph_keys, dim3(gn), dim3(256), 0, s, Na, vals, a.node_graph, a.rank,
                       sc.g0.p);
    bool alt2 = false;
    radix_sort_u32(sc.g0.p, vals, sc.g1.p, vals_alt, Na, gbits, sc.tmp.p, sc.tmp.bytes(), &alt2, s);
    const uint32_t *asc = alt2 ? vals_alt : vals;
    hipLaunchKernelGGL(k_batch_positions, dim3(gn), dim3(256), 0, s, Na, asc, sc.pos.p);
    const size_t hist_lds = (size_t)a.max_nodes * sizeof(uint32_t);
    if (a.edge_ptr && a.max_nodes > 0 && hist_lds <= kGraphHistLds) {
        if (hist_lds > 64 * 1024)
            LOWD_HIP(hipFuncSetAttribute((const void *)k_edge_min_pos_graph,
                                         hipFuncAttributeMaxDynamicSharedMemorySize,
                                         (int)hist_lds));
        hipLaunchKernelGGL(k_edge_min_pos_graph, dim3((unsigned)a.A), dim3(kGraphHistBlock),
                           hist_lds, s, a.act, a.seg, a.edge_ptr, a.gsrc, a.gdst, sc.pos.p,
                           (unsigned long long *)sc.hist.p);
    } else {
        hipLaunchKernelGGL(k_fill_i64, dim3(gn), dim3(256), 0, s, Na, sc.hist.p);
        if (a.M > 0)
            hipLaunchKernelGGL(k_edge_min_pos_batch, dim3(grid_for(a.M, 256)), dim3(256), 0, s,
                               a.M, a.gsrc, a.gdst, a.node_graph, a.rank, sc.pos.p,
                               (unsigned long long *)sc.hist.p);
    }
    hipLaunchKernelGGL(k_reverse<int64_t>, dim3(gn), dim3(256), 0, s, Na, sc.hist.p, sc.rev.p);
    exclusive_scan_i64(sc.rev.p, sc.rev.p, Na, nullptr, sc.tmp.p, sc.tmp.bytes(), s);
    hipLaunchKernelGGL(k_suffix<int64_t>, dim3(gn), dim3(256), 0, s, Na, sc.rev.p, sc.hist.p,
                       sc.W.p);
    hipLaunchKernelGGL(k_best_batch, dim3((unsigned)a.A), dim3(kArgBlock), 0, s, a.A, a.act,
                       a.seg, a.node_ptr, Na, sc.W.p, a.L64, sc.best.p, a.num, a.den, a.D);
    hipLaunchKernelGGL(k_in_set_batch, dim3(ga), dim3(256), 0, s, a.A, a.act, a.seg, a.node_ptr,
                       sc.pos.p, sc.best.p, a.in_set);
    LOWD_HIP(hipGetLastError());
}

namespace {
__global__ void k_entry_weights(int64_t len, const uint32_t *inc, const uint64_t *wi,
                                uint64_t *wi_inc) {
    for (int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; j < len;
         j += (int64_t)gridDim.x * blockDim.x)
        wi_inc[j] = wi[inc[j] >> 1];
}
}  // namespace

void build_entry_weights(int64_t m, const uint32_t *inc, const uint64_t *wi, uint64_t *wi_inc,
                         hipStream_t s) {
    if (m <= 0) return;
    hipLaunchKernelGGL(k_entry_weights, dim3(grid_for(2 * m, 256)), dim3(256), 0, s, 2 * m, inc,
                       wi, wi_inc);
    LOWD_HIP(hipGetLastError());
}

}  // namespace lowd
