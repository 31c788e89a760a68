// k_prune.hip -- Algorithm 2 (Pruning) for unweighted graphs.
//
// Section III-D prunes in O(M + N) with a counting sort of the nodes by
// degree: a round removes every node whose degree is below the current
// density delta = |E(H)| / |V(H)|, and the nodes of the first round are
// exactly a prefix of the degree-sorted order.  On the GPU:
//   1. degrees: one stable radix pass groups the edges' ends by the top
//      eight bits of the node id, then a workgroup counts a range of at
//      most 32K node ids in LDS; an LDS-privatised degree histogram (4096
//      bins, the last one collecting larger degrees) and a wave-scan
//      exclusive prefix give the bucket starts; a scatter sorts the nodes by
//      degree bucket;
//   2. round 1 removes the bucket prefix below delta without looking at the
//      other nodes; the surviving suffix becomes the alive list;
//   3. every later round tests the alive list (deg * |V(H)| < |E(H)|, exact
//      in int64) and splits it with two prefix sums into the removed list
//      and the next alive list;
//   4. each round then walks the list of H's edges once: an edge with a
//      removed end leaves H and lowers its other end's degree, the others
//      form the next, shorter list (|E(H)| is its length);
//   5. the kept nodes are renumbered by a prefix sum (ascending original id)
//      and the kept edges compacted by another, in their original order.
// The alive list shrinks quickly (the number of removed nodes decays
// exponentially, as the paper observes), so the rounds after the first cost
// little.
#include <cmath>
#include <vector>

#include <array>

#include "lowd_internal.h"
#include "prune.h"

namespace lowd {
namespace {

constexpr int kBins = 4096;

// Counts of node ids in [lo, lo + span) of one digit group: the group's ids
// in two partitioned id arrays (ids in ka grouped by v >> gshift with group
// starts sa, likewise kb and sb), counted in LDS.  Workgroup g takes group
// g / (S * P), id range (g / P) % S of it, and piece g % P of the group's
// ids.  The counts are stored in deg (sub = false) or taken off it (sub =
// true); with P = 1 a workgroup owns its ids and writes them plainly,
// otherwise it adds or subtracts with atomics (deg zeroed before, when
// storing).
constexpr int kCountBlock = 1024;
__device__ __forceinline__ void count_id(uint32_t *cnt, uint32_t v, int64_t lo, int64_t hi) {
    if ((int64_t)v >= lo && (int64_t)v < hi) atomicAdd(&cnt[(int64_t)v - lo], 1u);
}
constexpr int kCountBits = 15;   // at most 32K ids counted by a workgroup (128 KB of LDS)
__global__ void __launch_bounds__(kCountBlock)
k_count_ids(int32_t n, const uint32_t *ka, const int64_t *sa, const uint32_t *kb,
            const int64_t *sb, int gshift, int span_bits, int32_t S, int32_t P, bool sub,
            int32_t *deg) {
    extern __shared__ uint32_t cnt[];
    const int32_t g = (int32_t)blockIdx.x;
    const int32_t grp = g / (S * P), r = (g / P) % S, piece = g % P;
    const int64_t lo = ((int64_t)grp << gshift) + ((int64_t)r << span_bits);
    const int64_t span = (int64_t)1 << span_bits;
    const int64_t hi = lo + span < (int64_t)n ? lo + span : (int64_t)n;
    if (lo >= hi) return;   // uniform across the block
    for (int64_t i = threadIdx.x; i < span; i += kCountBlock) cnt[i] = 0;
    __syncthreads();
    for (int side = 0; side < 2; ++side) {
        const uint32_t *keys = side ? kb : ka;
        const int64_t *st = side ? sb : sa;
        const int64_t b = st[grp], len = st[grp + 1] - b;
        const int64_t p0 = b + len * piece / P, p1 = b + len * (piece + 1) / P;
        // 16-byte loads, four in flight a lane, from the first 16-byte
        // aligned key on; the ends one key at a time
        const int64_t skip = (int64_t)((4u - (uint32_t)(((uintptr_t)(keys + p0) & 15u) >> 2)) & 3u);
        const int64_t a0 = p0 + skip < p1 ? p0 + skip : p1;
        const int64_t a1 = a0 + ((p1 - a0) & ~(int64_t)3);
        for (int64_t i = p0 + threadIdx.x; i < a0; i += kCountBlock) count_id(cnt, keys[i], lo, hi);
        for (int64_t i = a1 + threadIdx.x; i < p1; i += kCountBlock) count_id(cnt, keys[i], lo, hi);
        constexpr int kU = 4;
        const uint4 *vk = reinterpret_cast<const uint4 *>(keys + a0);
        const int64_t nv = (a1 - a0) / 4;
        for (int64_t j = threadIdx.x; j < nv; j += (int64_t)kU * kCountBlock) {
            uint4 q[kU];
#pragma unroll
            for (int u = 0; u < kU; ++u)
                q[u] = j + u * kCountBlock < nv ? vk[j + u * kCountBlock]
                                                : make_uint4(~0u, ~0u, ~0u, ~0u);
#pragma unroll
            for (int u = 0; u < kU; ++u) {
                count_id(cnt, q[u].x, lo, hi);
                count_id(cnt, q[u].y, lo, hi);
                count_id(cnt, q[u].z, lo, hi);
                count_id(cnt, q[u].w, lo, hi);
            }
        }
    }
    __syncthreads();
    for (int64_t i = threadIdx.x; i < hi - lo; i += kCountBlock) {
        const int32_t c = (int32_t)cnt[i];
        if (P == 1) {
            if (!sub) deg[lo + i] = c;
            else if (c) deg[lo + i] -= c;
        } else if (c) {
            if (sub) atomicSub(&deg[lo + i], c);
            else atomicAdd(&deg[lo + i], c);
        }
    }
}

__global__ void __launch_bounds__(256) k_degree_hist(int32_t n, const int32_t *deg,
                                                     unsigned long long *hist) {
    __shared__ uint32_t h[kBins];
    for (int b = threadIdx.x; b < kBins; b += blockDim.x) h[b] = 0;
    __syncthreads();
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x) {
        int32_t d = deg[u];
        atomicAdd(&h[d < kBins - 1 ? d : kBins - 1], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kBins; b += blockDim.x)
        if (h[b]) atomicAdd(&hist[b], (unsigned long long)h[b]);
}

// The counting sort's scatter.  Block b places the nodes of its chunk
// [b * kScatterChunk, (b + 1) * kScatterChunk): it counts them per bin in
// LDS, reserves each non-empty bin's range with one global atomic, then
// ranks the nodes inside the range with LDS atomics.  (A global atomic per
// node serialises on the few bins that hold most nodes.)  The order inside
// a bin is arbitrary; nothing downstream depends on it.
constexpr int kScatterBlock = 256;
constexpr int64_t kScatterChunk = 16 * kScatterBlock;
__global__ void __launch_bounds__(kScatterBlock)
k_bucket_scatter(int32_t n, const int32_t *deg, const int64_t *bin_start,
                 unsigned long long *cursor, int32_t *by_deg) {
    __shared__ uint32_t cnt[kBins];
    __shared__ int64_t base[kBins];
    for (int b = threadIdx.x; b < kBins; b += kScatterBlock) cnt[b] = 0;
    __syncthreads();
    const int64_t lo = (int64_t)blockIdx.x * kScatterChunk;
    const int64_t hi = lo + kScatterChunk < n ? lo + kScatterChunk : (int64_t)n;
    for (int64_t u = lo + threadIdx.x; u < hi; u += kScatterBlock) {
        const int32_t d = deg[u];
        atomicAdd(&cnt[d < kBins - 1 ? d : kBins - 1], 1u);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < kBins; b += kScatterBlock) {
        const uint32_t c = cnt[b];
        base[b] = c ? bin_start[b] + (int64_t)atomicAdd(&cursor[b], (unsigned long long)c) : 0;
        cnt[b] = 0;
    }
    __syncthreads();
    for (int64_t u = lo + threadIdx.x; u < hi; u += kScatterBlock) {
        const int32_t d = deg[u];
        const int b = d < kBins - 1 ? d : kBins - 1;
        by_deg[base[b] + (int64_t)atomicAdd(&cnt[b], 1u)] = (int32_t)u;
    }
}

// flags for the split of a candidate list into removed / kept
__global__ void k_test(int64_t c, const int32_t *cand, const int32_t *deg, int64_t N, int64_t M,
                       int64_t *rm, int64_t *keep) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < c;
         i += (int64_t)gridDim.x * blockDim.x) {
        bool r = (int64_t)deg[cand[i]] * N < M;
        rm[i] = r ? 1 : 0;
        keep[i] = r ? 0 : 1;
    }
}

__global__ void k_split(int64_t c, const int32_t *cand, const int64_t *rm, const int64_t *rm_pos,
                        const int64_t *keep_pos, int32_t *removed, int32_t *alive) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < c;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (rm[i]) removed[rm_pos[i]] = cand[i];
        else alive[keep_pos[i]] = cand[i];
    }
}

// stamp[v]: 0 for an alive node, -(slot + 1) for an alive hub (below), r > 0
// once removed in round r.
// The kHubs highest-degree nodes (the tail of the degree-bucketed order) are
// hubs: the round kernel counts their lost edges per workgroup in LDS and
// adds each count with one atomic, where the rounds' removed edges would
// otherwise send one atomic each to the same few degree counters.
constexpr int kHubs = 4096;

// The round kernel reads an end's state from 2-bit marks, 16 nodes a word
// (4 MB for 16M nodes, about an L2's size, where the stamps take 64 MB and
// every read of one would go past the L2): dead, alive, removed in the
// current round, alive hub.
constexpr uint32_t kMarkDead = 0u, kMarkAlive = 1u, kMarkNow = 2u, kMarkHub = 3u;
__device__ __forceinline__ uint32_t mark_of(const uint32_t *marks, int32_t v) {
    return (marks[v >> 4] >> ((v & 15) * 2)) & 3u;
}

__global__ void k_mark_hubs(int32_t k, const int32_t *hubs, int32_t *stamp) {
    for (int32_t i = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x); i < k;
         i += (int32_t)(gridDim.x * blockDim.x))
        stamp[hubs[i]] = -(i + 1);
}

__global__ void k_stamp(int64_t k, const int32_t *list, int32_t *stamp, int32_t round) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * blockDim.x)
        stamp[list[i]] = round;
}

// The marks from the stamps in one pass (round 0: alive, hubs and dead
// only): each lane finds its node's mark and 16 lanes OR theirs into one
// word.  Every lane of a wave runs the same iterations (the loop bound is
// uniform), so the shuffles see whole waves.
__global__ void k_marks(int32_t n, const int32_t *stamp, uint32_t *marks, int32_t round) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += stride) {
        const int64_t v = base + threadIdx.x;
        uint32_t mk = kMarkDead;
        if (v < n) {
            const int32_t st = stamp[v];
            mk = st == 0 ? kMarkAlive : st < 0 ? kMarkHub : st == round ? kMarkNow : kMarkDead;
        }
        uint32_t word = mk << ((uint32_t)(v & 15) * 2);
        for (int o = 1; o < 16; o <<= 1) word |= __shfl_xor(word, o, kWave);
        if ((v & 15) == 0 && v < n) marks[v >> 4] = word;
    }
}

// One round over H's edge list (the original src/dst arrays in the first
// round, packed (src, dst) pairs after it): every edge whose ends are both
// still alive goes to the next list; every other one leaves H and its end
// that stays loses a degree: a hub's loss is counted per workgroup in LDS
// and added once at the end, any other end is written to the list of
// decrements (counted by node afterwards, where an atomic per edge on the
// degrees ran at about 14 G/s).  The list's ends are all alive when the
// round starts, so a mark here is alive, hub or removed now.  A tile of
// kRoundRows rows of 256 edges loads its ends and then their marks, all in
// flight together; its kept edges and its decrements each take one range of
// their list with one atomic, ranked by wave ballots (the order within the
// lists does not matter: H's final edge list is compacted from the original
// arrays).
constexpr int kRoundBlock = 256, kRoundRows = 16;
constexpr int kRoundWaves = kRoundBlock / kWave;
constexpr int64_t kRoundTile = (int64_t)kRoundBlock * kRoundRows;
constexpr int64_t kRoundGrid = 1024;
__global__ void __launch_bounds__(kRoundBlock)
k_prune_round(int64_t k, const int32_t *src, const int32_t *dst, const uint2 *in,
              const uint32_t *marks, const int32_t *stamp, int32_t *deg, const int32_t *hubs,
              int32_t nhubs, uint2 *out, uint32_t *dec, unsigned long long *counts) {
    __shared__ int32_t hub_lost[kHubs];
    __shared__ int wcnt[2][kRoundRows][kRoundWaves];
    __shared__ unsigned long long tile_base[2];
    for (int i = threadIdx.x; i < kHubs; i += kRoundBlock) hub_lost[i] = 0;
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    const int64_t ntiles = (k + kRoundTile - 1) / kRoundTile;
    __syncthreads();
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {   // uniform across the block
        int32_t a[kRoundRows], b[kRoundRows];
        uint32_t ma[kRoundRows], mb[kRoundRows];
        uint64_t bal[kRoundRows], dbal[kRoundRows];
#pragma unroll
        for (int q = 0; q < kRoundRows; ++q) {
            const int64_t e = t * kRoundTile + (int64_t)q * kRoundBlock + threadIdx.x;
            a[q] = -1;
            b[q] = -1;
            if (e < k) {
                if (in) {
                    const uint2 pr = in[e];
                    a[q] = (int32_t)pr.x;
                    b[q] = (int32_t)pr.y;
                } else {
                    a[q] = src[e];
                    b[q] = dst[e];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < kRoundRows; ++q) {
            ma[q] = a[q] >= 0 ? mark_of(marks, a[q]) : kMarkDead;
            mb[q] = b[q] >= 0 ? mark_of(marks, b[q]) : kMarkDead;
        }
#pragma unroll
        for (int q = 0; q < kRoundRows; ++q) {
            // alive and hub marks have the low bit, removed-now does not
            const bool valid = a[q] >= 0;
            const bool stays = valid && ((ma[q] & mb[q] & 1u) != 0);
            const bool a_left = (ma[q] & 1u) != 0, b_left = (mb[q] & 1u) != 0;
            const bool loses = valid && !stays && (a_left || b_left);
            const uint32_t mv = a_left ? ma[q] : mb[q];
            // the end that stays, kept in a[q] for the decrement list
            if (loses && !a_left) a[q] = b[q];
            if (loses && mv == kMarkHub) atomicAdd(&hub_lost[-stamp[a[q]] - 1], 1);   // its slot
            bal[q] = __ballot(stays);
            dbal[q] = __ballot(loses && mv != kMarkHub);
            if (lane == 0) {
                wcnt[0][q][wave] = __popcll(bal[q]);
                wcnt[1][q][wave] = __popcll(dbal[q]);
            }
        }
        __syncthreads();
        if (threadIdx.x < 2) {
            int total = 0;
            for (int q = 0; q < kRoundRows; ++q)
                for (int w = 0; w < kRoundWaves; ++w) total += wcnt[threadIdx.x][q][w];
            tile_base[threadIdx.x] =
                total ? atomicAdd(&counts[threadIdx.x], (unsigned long long)total) : 0ull;
        }
        __syncthreads();
        unsigned long long base = tile_base[0], dbase = tile_base[1];
#pragma unroll
        for (int q = 0; q < kRoundRows; ++q) {
            int before = 0, row = 0, dbefore = 0, drow = 0;
            for (int w = 0; w < kRoundWaves; ++w) {
                before += w < wave ? wcnt[0][q][w] : 0;
                row += wcnt[0][q][w];
                dbefore += w < wave ? wcnt[1][q][w] : 0;
                drow += wcnt[1][q][w];
            }
            if ((bal[q] >> lane) & 1ull)
                out[base + (unsigned long long)(before + __popcll(bal[q] & lt))] =
                    make_uint2((uint32_t)a[q], (uint32_t)b[q]);
            if ((dbal[q] >> lane) & 1ull)
                dec[dbase + (unsigned long long)(dbefore + __popcll(dbal[q] & lt))] =
                    (uint32_t)a[q];
            base += (unsigned long long)row;
            dbase += (unsigned long long)drow;
        }
        __syncthreads();   // wcnt and tile_base are reused by the next tile
    }
    for (int i = threadIdx.x; i < nhubs; i += kRoundBlock) {
        const int32_t c = hub_lost[i];
        if (c) atomicSub(&deg[hubs[i]], c);
    }
}

__global__ void k_keep_flags(int32_t n, const int32_t *stamp, uint8_t *node_keep, int64_t *flag) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x) {
        bool k = stamp[u] <= 0;
        node_keep[u] = k ? 1 : 0;
        flag[u] = k ? 1 : 0;
    }
}

__global__ void k_relabel(int32_t n, const int64_t *flag, const int64_t *pos, int32_t *relabel) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < n;
         u += (int64_t)gridDim.x * blockDim.x)
        relabel[u] = flag[u] ? (int32_t)pos[u] : -1;
}

// The edges of H (both ends kept), compacted in their original order, in
// two passes over tiles of kCompactTile edges, each a block of 256 threads
// reading rows of 256 consecutive edges: the first marks each edge and
// counts a tile's kept edges; after a scan of the tile counts, the second
// writes a tile's kept edges from its offset, ranked within each row by a
// wave ballot (rows in order, waves in order within a row).
constexpr int kCompactBlock = 256, kCompactRows = 16;
constexpr int kCompactWaves = kCompactBlock / kWave;
constexpr int64_t kCompactTile = (int64_t)kCompactBlock * kCompactRows;

__global__ void __launch_bounds__(kCompactBlock)
    k_edge_keep_tiles(int64_t m, const int32_t *src, const int32_t *dst, const int32_t *stamp,
                      const uint32_t *marks, uint8_t *keep, int64_t *tile_count) {
    __shared__ int lds[kCompactWaves];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const int64_t ntiles = (m + kCompactTile - 1) / kCompactTile;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {   // uniform across the block
        // the tile's ends first, all loads in flight, then their states
        int32_t a[kCompactRows], b[kCompactRows];
        bool kp[kCompactRows];
#pragma unroll
        for (int k = 0; k < kCompactRows; ++k) {
            const int64_t e = t * kCompactTile + (int64_t)k * kCompactBlock + threadIdx.x;
            a[k] = e < m ? src[e] : 0;
            b[k] = e < m ? dst[e] : 0;
        }
#pragma unroll
        for (int k = 0; k < kCompactRows; ++k)   // kept: both ends alive (alive and hub
            kp[k] = marks                         // marks have the low bit)
                        ? ((mark_of(marks, a[k]) & mark_of(marks, b[k]) & 1u) != 0)
                        : (stamp[a[k]] <= 0 && stamp[b[k]] <= 0);
        int c = 0;
#pragma unroll
        for (int k = 0; k < kCompactRows; ++k) {
            const int64_t e = t * kCompactTile + (int64_t)k * kCompactBlock + threadIdx.x;
            if (e < m) {
                keep[e] = kp[k] ? 1 : 0;
                c += kp[k] ? 1 : 0;
            }
        }
        for (int d = kWave / 2; d > 0; d >>= 1) c += __shfl_down(c, d, kWave);
        if (lane == 0) lds[wave] = c;
        __syncthreads();
        if (threadIdx.x == 0) {
            int total = 0;
            for (int w = 0; w < kCompactWaves; ++w) total += lds[w];
            tile_count[t] = total;
        }
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kCompactBlock)
    k_edge_write_tiles(int64_t m, const int32_t *src, const int32_t *dst, const float *w,
                       const uint8_t *keep, const int64_t *tile_offset, const int64_t *npos,
                       int32_t *h_src, int32_t *h_dst, float *h_w, int64_t *edge_map) {
    __shared__ int cnt[kCompactRows][kCompactWaves];
    const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
    const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (kWave - lane));
    const int64_t ntiles = (m + kCompactTile - 1) / kCompactTile;
    for (int64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {   // uniform across the block
        uint64_t ball[kCompactRows];
        for (int k = 0; k < kCompactRows; ++k) {
            const int64_t e = t * kCompactTile + (int64_t)k * kCompactBlock + threadIdx.x;
            ball[k] = __ballot(e < m && keep[e] != 0);
            if (lane == 0) cnt[k][wave] = __popcll(ball[k]);
        }
        __syncthreads();
        int64_t base = tile_offset[t];
        for (int k = 0; k < kCompactRows; ++k) {
            int before = 0, row = 0;
            for (int v = 0; v < kCompactWaves; ++v) {
                before += v < wave ? cnt[k][v] : 0;
                row += cnt[k][v];
            }
            if ((ball[k] >> lane) & 1ull) {
                const int64_t e = t * kCompactTile + (int64_t)k * kCompactBlock + threadIdx.x;
                const int64_t at = base + before + __popcll(ball[k] & lt);
                if (h_src) {
                    h_src[at] = (int32_t)npos[src[e]];
                    h_dst[at] = (int32_t)npos[dst[e]];
                }
                if (h_w) h_w[at] = w[e];
                if (edge_map) edge_map[at] = e;
            }
            base += row;
        }
        __syncthreads();
    }
}

// buffers of compact_edges for m edges
inline int64_t compact_tiles(int64_t m) { return (m + kCompactTile - 1) / kCompactTile; }

// H's edge list (renumbered by npos) from the kept flags of the nodes
// (stamp <= 0, or from the marks where given: their 4 MB stay in the L2
// where the stamps' 64 MB do not); *kept_dev (device) receives the number
// of H's edges.
void compact_edges(int64_t m, const int32_t *src, const int32_t *dst, const float *w,
                   const int32_t *stamp, const uint32_t *marks, const int64_t *npos,
                   int32_t *h_src, int32_t *h_dst,
                   float *h_w, int64_t *edge_map, uint8_t *keep, int64_t *tile_count,
                   int64_t *tile_offset, int64_t *kept_dev, void *scan_tmp, size_t scan_bytes,
                   hipStream_t s) {
    if (m <= 0) return;
    const int64_t nt = compact_tiles(m);
    const unsigned g = (unsigned)std::min<int64_t>(nt, 65536);
    hipLaunchKernelGGL(k_edge_keep_tiles, dim3(g), dim3(kCompactBlock), 0, s, m, src, dst, stamp,
                       marks, keep, tile_count);
    exclusive_scan_i64(tile_count, tile_offset, nt, kept_dev, scan_tmp, scan_bytes, s);
    if (h_src || h_w || edge_map)
        hipLaunchKernelGGL(k_edge_write_tiles, dim3(g), dim3(kCompactBlock), 0, s, m, src, dst, w,
                           keep, tile_offset, npos, h_src, h_dst, h_w, edge_map);
    LOWD_HIP(hipGetLastError());
}

// ------------------------------------------------------ weighted graphs --
// Algorithm 2 with weighted degrees (Section III-D: every round scans the
// nodes still alive).  The test deg_w(u) < rho(H) = w(E(H)) / |V(H)| is
// decided exactly.  Every float32 weight is m * 2^q with an integer m <
// 2^24; with q_min the smallest such q over the edges, w / 2^q_min is an
// integer, below 2^64 when the exponents span at most 40 binades.  Degrees
// and 2 w(E(H)) = sum of degrees are then exact 128-bit sums in any order,
// and 2 deg(u) |V(H)| < 2 w(E(H)) an exact 128-bit comparison.

__device__ __forceinline__ int32_t ulp_exponent(float x) {
    const uint32_t b = __builtin_bit_cast(uint32_t, x);
    const int32_t e = (int32_t)((b >> 23) & 0xFFu);
    return e == 0 ? -149 : e - 150;
}
__device__ __forceinline__ uint64_t significand(float x) {
    const uint32_t b = __builtin_bit_cast(uint32_t, x);
    const uint32_t f = b & 0x7FFFFFu;
    return ((b >> 23) & 0xFFu) == 0 ? (uint64_t)f : (uint64_t)(f | 0x800000u);
}

__global__ void k_exponent_range(int64_t m, const float *w, int32_t *range) {
    int32_t lo = 1 << 30, hi = -(1 << 30);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t q = ulp_exponent(w[e]);
        lo = q < lo ? q : lo;
        hi = q > hi ? q : hi;
    }
    for (int o = kWave / 2; o > 0; o >>= 1) {   // one atomic pair per wave
        const int32_t a = __shfl_down(lo, o, kWave), b = __shfl_down(hi, o, kWave);
        lo = a < lo ? a : lo;
        hi = b > hi ? b : hi;
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        atomicMin(&range[0], lo);
        atomicMax(&range[1], hi);
    }
}

__global__ void k_fixed_weights(int64_t m, const float *w, int32_t qmin, uint64_t *wi) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < m;
         e += (int64_t)gridDim.x * blockDim.x)
        wi[e] = significand(w[e]) << (ulp_exponent(w[e]) - qmin);
}

__global__ void k_iota(int32_t n, int32_t *a) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        a[i] = (int32_t)i;
}

__device__ __forceinline__ u128 shfl_down_u128(u128 v, int d) {
    const uint64_t lo = __shfl_down((uint64_t)v, d, kWave);
    const uint64_t hi = __shfl_down((uint64_t)(v >> 64), d, kWave);
    return ((u128)hi << 64) | lo;
}

// weighted degree in H of every alive node (one wavefront per node); the
// degree of list entry i goes to (dlo[i], dhi[i])
__global__ void __launch_bounds__(256) k_weighted_degrees(int64_t k, const int32_t *alive,
                                                          const int64_t *row_ptr,
                                                          const uint32_t *inc, const int32_t *src,
                                                          const int32_t *dst, const int32_t *stamp,
                                                          const uint64_t *wi, uint64_t *dlo,
                                                          uint64_t *dhi) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / kWave);
    for (int64_t i = (int64_t)blockIdx.x * (blockDim.x / kWave) + threadIdx.x / kWave; i < k;
         i += waves) {
        const int32_t u = alive[i];
        u128 acc = 0;
        for (int64_t j = row_ptr[u] + lane; j < row_ptr[u + 1]; j += kWave) {
            const uint32_t ent = inc[j];
            const int64_t e = ent >> 1;
            const int32_t v = (ent & 1) ? src[e] : dst[e];
            if (stamp[v] == 0) acc += (u128)wi[e];
        }
        for (int d = kWave / 2; d > 0; d >>= 1) acc += shfl_down_u128(acc, d);
        if (lane == 0) {
            dlo[i] = (uint64_t)acc;
            dhi[i] = (uint64_t)(acc >> 64);
        }
    }
}

// sum of the k degrees (exact; blocks write partials, then one block adds them)
constexpr int kSumBlock = 256;
__global__ void __launch_bounds__(kSumBlock) k_sum_u128(int64_t k, const uint64_t *lo,
                                                        const uint64_t *hi, uint64_t *out_lo,
                                                        uint64_t *out_hi) {
    __shared__ uint64_t sl[kSumBlock], sh[kSumBlock];
    u128 acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * blockDim.x)
        acc += ((u128)hi[i] << 64) | lo[i];
    sl[threadIdx.x] = (uint64_t)acc;
    sh[threadIdx.x] = (uint64_t)(acc >> 64);
    __syncthreads();
    for (int d = kSumBlock / 2; d > 0; d >>= 1) {
        if ((int)threadIdx.x < d) {
            const u128 a = ((u128)sh[threadIdx.x] << 64) | sl[threadIdx.x];
            const u128 b = ((u128)sh[threadIdx.x + d] << 64) | sl[threadIdx.x + d];
            const u128 c = a + b;
            sl[threadIdx.x] = (uint64_t)c;
            sh[threadIdx.x] = (uint64_t)(c >> 64);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out_lo[blockIdx.x] = sl[0];
        out_hi[blockIdx.x] = sh[0];
    }
}

// removal test of every alive node: 2 deg(u) N < sum of degrees (= 2 w(E(H)))
__global__ void k_weighted_test(int64_t k, const uint64_t *dlo, const uint64_t *dhi, int64_t N,
                                const uint64_t *total_lo, const uint64_t *total_hi, int64_t *rm,
                                int64_t *keep) {
    const u128 W2 = ((u128)total_hi[0] << 64) | total_lo[0];
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < k;
         i += (int64_t)gridDim.x * blockDim.x) {
        const u128 d = ((u128)dhi[i] << 64) | dlo[i];
        const bool r = d * (u128)(2 * N) < W2;
        rm[i] = r ? 1 : 0;
        keep[i] = r ? 0 : 1;
    }
}

}  // namespace

void fixed_point_weights(int64_t m, const float *w, uint64_t *wi, int32_t *q_out,
                         int32_t *range_dev, hipStream_t s) {
    *q_out = 0;
    if (m <= 0) return;
    const int32_t init[2] = {1 << 30, -(1 << 30)};
    LOWD_HIP(hipMemcpyAsync(range_dev, init, sizeof(init), hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_exponent_range, dim3(grid_for(m, 256, 1024)), dim3(256), 0, s, m, w,
                       range_dev);
    int32_t r[2];
    LOWD_HIP(hipMemcpyAsync(r, range_dev, sizeof(r), hipMemcpyDeviceToHost, s));
    LOWD_HIP(hipStreamSynchronize(s));
    if (r[1] - r[0] > kMaxExpSpan)
        fail(LOWD_E_UNSUPPORTED, "weights span more than 2^40 in scale; exact weighted sums need "
                                 "them closer");
    *q_out = r[0];
    hipLaunchKernelGGL(k_fixed_weights, dim3(grid_for(m, 256)), dim3(256), 0, s, m, w, r[0], wi);
    LOWD_HIP(hipGetLastError());
}

namespace {
__global__ void k_whole_group(int64_t m, int64_t *starts) {
    if (threadIdx.x == 0) {
        starts[0] = 0;
        starts[1] = m;
    }
}

// Buffers of count_ids for up to `cap` ids a side.
struct CountBufs {
    uint32_t *pa, *pb;     // the two sides grouped by digit
    int64_t *sa, *sb;      // group starts (257 each)
    char *tmp;             // radix pass scratch
    size_t tmp_bytes;
};
constexpr int kGroups = 256;
CountBufs take_count_bufs(int64_t cap, Arena &ws) {
    CountBufs c;
    const size_t k = (size_t)(cap > 0 ? cap : 1);
    c.pa = ws.take<uint32_t>(k);
    c.pb = ws.take<uint32_t>(k);
    c.sa = ws.take<int64_t>(kGroups + 1);
    c.sb = ws.take<int64_t>(kGroups + 1);
    c.tmp_bytes = radix_sort_tmp_bytes(cap);
    c.tmp = ws.take<char>(c.tmp_bytes);
    return c;
}

// deg[v] = (sub ? deg[v] - : ) the number of times v appears in a[0..na)
// and b[0..nb) (b may be empty).  Node ids of more than kCountBits bits are
// first grouped by their top eight bits (a stable radix pass over each
// side), so that every workgroup of k_count_ids reads only the ids of its
// group; a group's ids are split into pieces where one would exceed
// kPieceIds.  Neither a nor b may lie in c.pa or c.pb.
constexpr int64_t kPieceIds = (int64_t)1 << 22;
void count_ids(int32_t n, const uint32_t *a, int64_t na, const uint32_t *b, int64_t nb,
               int32_t *deg, bool sub, const CountBufs &c, hipStream_t s) {
    if (n <= 0) return;
    int bits = 1;
    while (bits < 31 && ((int64_t)1 << bits) < (int64_t)n) ++bits;
    const bool grouped = bits > kCountBits;
    const int gshift = grouped ? bits - 8 : 0;
    const int span_bits = grouped ? std::min(gshift, kCountBits) : bits;
    const int32_t S = grouped ? (int32_t)1 << (gshift - span_bits) : 1;
    const int32_t ngroups = grouped ? kGroups : 1;
    if (grouped) {
        radix_partition_u32(a, c.pa, na, gshift, c.sa, c.tmp, c.tmp_bytes, s);
        radix_partition_u32(b, c.pb, nb, gshift, c.sb, c.tmp, c.tmp_bytes, s);
    } else {
        hipLaunchKernelGGL(k_whole_group, dim3(1), dim3(1), 0, s, na, c.sa);
        hipLaunchKernelGGL(k_whole_group, dim3(1), dim3(1), 0, s, nb, c.sb);
    }
    std::vector<int64_t> ha((size_t)kGroups + 1), hb((size_t)kGroups + 1);
    LOWD_HIP(hipMemcpyAsync(ha.data(), c.sa, (size_t)(ngroups + 1) * sizeof(int64_t),
                            hipMemcpyDeviceToHost, s));
    LOWD_HIP(hipMemcpyAsync(hb.data(), c.sb, (size_t)(ngroups + 1) * sizeof(int64_t),
                            hipMemcpyDeviceToHost, s));
    LOWD_HIP(hipStreamSynchronize(s));
    int64_t most = 0;
    for (int32_t g = 0; g < ngroups; ++g)
        most = std::max<int64_t>(most, ha[g + 1] - ha[g] + hb[g + 1] - hb[g]);
    const int32_t P = (int32_t)std::min<int64_t>(
        std::max<int64_t>((most + kPieceIds - 1) / kPieceIds, 1), 256);
    if (P > 1 && !sub) LOWD_HIP(hipMemsetAsync(deg, 0, (size_t)n * sizeof(int32_t), s));
    const size_t lds = ((size_t)1 << span_bits) * sizeof(uint32_t);
    LOWD_HIP(hipFuncSetAttribute((const void *)k_count_ids,
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    hipLaunchKernelGGL(k_count_ids, dim3((unsigned)((int64_t)ngroups * S * P)), dim3(kCountBlock),
                       lds, s, n, grouped ? c.pa : a, c.sa, grouped ? c.pb : b, c.sb, gshift,
                       span_bits, S, P, sub, deg);
    LOWD_HIP(hipGetLastError());
}
}  // namespace

// Every device buffer of the prune comes from `ws`, taken in a fixed order,
// so a region without a base measures what a call needs (prune_ws_bytes).
PruneResult run_prune_ws(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                         uint8_t *node_keep, int32_t *relabel, int32_t *h_src, int32_t *h_dst,
                         int64_t *edge_map, Arena &ws, hipStream_t s) {
    PruneResult res;
    const unsigned gn = grid_for(n, 256);
    const size_t nn = (size_t)n;
    int32_t *deg = ws.take<int32_t>(nn);
    const CountBufs cb = take_count_bufs(m, ws);
    uint32_t *dec = ws.take<uint32_t>((size_t)(m > 0 ? m : 1));   // a round's decrements
    uint32_t *marks = ws.take<uint32_t>((nn + 15) / 16);
    int32_t *stamp = ws.take<int32_t>(nn), *by_deg = ws.take<int32_t>(nn),
            *list_a = ws.take<int32_t>(nn), *list_b = ws.take<int32_t>(nn),
            *removed = ws.take<int32_t>(nn);
    unsigned long long *hist = ws.take<unsigned long long>(kBins),
                       *cursor = ws.take<unsigned long long>(kBins),
                       *counts = ws.take<unsigned long long>(2);
    int64_t *bin_start = ws.take<int64_t>(kBins), *f_rm = ws.take<int64_t>(nn),
            *f_keep = ws.take<int64_t>(nn), *p_rm = ws.take<int64_t>(nn),
            *p_keep = ws.take<int64_t>(nn), *tot = ws.take<int64_t>(2);
    // H's edge list between rounds, twice (the rounds alternate)
    uint2 *elist[2] = {ws.take<uint2>((size_t)(m > 0 ? m : 1)),
                       ws.take<uint2>((size_t)(m > 0 ? m : 1))};
    int64_t big = std::max<int64_t>(std::max<int64_t>(n, compact_tiles(m)), kBins);
    const size_t scan_bytes = exclusive_scan_tmp_bytes(big);
    char *scan_tmp = ws.take<char>(scan_bytes);
    const bool edges_out = (h_src || edge_map) && m > 0;
    const int64_t nt = compact_tiles(m);
    uint8_t *ekeep = edges_out ? ws.take<uint8_t>((size_t)m) : nullptr;
    int64_t *tcount = edges_out ? ws.take<int64_t>((size_t)nt) : nullptr;
    int64_t *toff = edges_out ? ws.take<int64_t>((size_t)nt + 1) : nullptr;
    if (!ws.base) return res;   // measuring only

    count_ids(n, (const uint32_t *)src, m, (const uint32_t *)dst, m, deg, false, cb, s);
    LOWD_HIP(hipMemsetAsync(hist, 0, kBins * sizeof(unsigned long long), s));
    LOWD_HIP(hipMemsetAsync(cursor, 0, kBins * sizeof(unsigned long long), s));
    LOWD_HIP(hipMemsetAsync(stamp, 0, (size_t)n * sizeof(int32_t), s));
    hipLaunchKernelGGL(k_degree_hist, dim3(grid_for(n, 256, 1024)), dim3(256), 0, s, n, deg,
                       hist);
    exclusive_scan_i64((const int64_t *)hist, bin_start, kBins, nullptr, scan_tmp, scan_bytes, s);
    if (n > 0)
        hipLaunchKernelGGL(k_bucket_scatter, dim3((unsigned)((n + kScatterChunk - 1) / kScatterChunk)),
                           dim3(kScatterBlock), 0, s, n, deg, bin_start, cursor, by_deg);
    const int32_t nhubs = n < kHubs ? n : kHubs;
    const int32_t *hubs = by_deg + (n - nhubs);   // the highest degrees
    if (nhubs > 0)
        hipLaunchKernelGGL(k_mark_hubs, dim3(grid_for(nhubs, 256)), dim3(256), 0, s, nhubs, hubs,
                           stamp);
    hipLaunchKernelGGL(k_marks, dim3(gn), dim3(256), 0, s, n, stamp, marks, 0);
    std::array<int64_t, kBins> hstart;
    LOWD_HIP(hipMemcpyAsync(hstart.data(), bin_start, kBins * sizeof(int64_t),
                            hipMemcpyDeviceToHost, s));
    LOWD_HIP(hipStreamSynchronize(s));

    int64_t N = n, M = m;
    const int32_t *alive = by_deg;   // current alive list (read only)
    int64_t nalive = n;
    for (int32_t round = 1;; ++round) {
        const int32_t *rm_list;
        int64_t nrm;
        if (round == 1 && M > 0 && (M + N - 1) / N <= kBins - 1) {
            // the removed nodes are the buckets of degree < ceil(M / N)
            int64_t cut = hstart[(size_t)((M + N - 1) / N)];
            rm_list = by_deg;
            nrm = cut;
            alive = by_deg + cut;
            nalive = n - cut;
        } else {
            if (nalive == 0 || M == 0) break;
            const unsigned gc = grid_for(nalive, 256);
            hipLaunchKernelGGL(k_test, dim3(gc), dim3(256), 0, s, nalive, alive, deg, N, M,
                               f_rm, f_keep);
            exclusive_scan_i64(f_rm, p_rm, nalive, tot, scan_tmp, scan_bytes, s);
            exclusive_scan_i64(f_keep, p_keep, nalive, tot + 1, scan_tmp, scan_bytes,
                               s);
            int32_t *out = (alive == list_a) ? list_b : list_a;
            hipLaunchKernelGGL(k_split, dim3(gc), dim3(256), 0, s, nalive, alive, f_rm, p_rm,
                               p_keep, removed, out);
            int64_t t[2];
            LOWD_HIP(hipMemcpyAsync(t, tot, sizeof(t), hipMemcpyDeviceToHost, s));
            LOWD_HIP(hipStreamSynchronize(s));
            rm_list = removed;
            nrm = t[0];
            alive = out;
            nalive = t[1];
        }
        if (nrm == 0) break;
        LOWD_HIP(hipMemsetAsync(counts, 0, 2 * sizeof(unsigned long long), s));
        const unsigned gr = grid_for(nrm, 256);
        hipLaunchKernelGGL(k_stamp, dim3(gr), dim3(256), 0, s, nrm, rm_list, stamp, round);
        hipLaunchKernelGGL(k_marks, dim3(gn), dim3(256), 0, s, n, stamp, marks, round);
        // at most kRoundGrid workgroups, each over many tiles, so that the
        // hubs' LDS counts are added with few atomics
        const uint2 *in = round == 1 ? nullptr : elist[round & 1];
        uint2 *out = elist[(round + 1) & 1];
        hipLaunchKernelGGL(k_prune_round, dim3(grid_for(M, (int)kRoundTile, kRoundGrid)),
                           dim3(kRoundBlock), 0, s, M, src, dst, in, marks, stamp, deg, hubs,
                           nhubs, out, dec, counts);
        LOWD_HIP(hipGetLastError());
        unsigned long long c[2] = {0, 0};
        LOWD_HIP(hipMemcpyAsync(c, counts, sizeof(c), hipMemcpyDeviceToHost, s));
        LOWD_HIP(hipStreamSynchronize(s));
        if (c[1] > 0) count_ids(n, dec, (int64_t)c[1], nullptr, 0, deg, true, cb, s);
        N -= nrm;
        M = (int64_t)c[0];
        res.rounds = round;
    }

    // outputs: mask, renumbering, compacted edge list
    hipLaunchKernelGGL(k_keep_flags, dim3(gn), dim3(256), 0, s, n, stamp, node_keep, f_keep);
    exclusive_scan_i64(f_keep, p_keep, n, nullptr, scan_tmp, scan_bytes, s);
    if (relabel)
        hipLaunchKernelGGL(k_relabel, dim3(gn), dim3(256), 0, s, n, f_keep, p_keep, relabel);
    if (edges_out) {
        compact_edges(m, src, dst, nullptr, stamp, marks, p_keep, h_src, h_dst, nullptr,
                      edge_map, ekeep, tcount, toff, toff + nt, scan_tmp, scan_bytes, s);
        LOWD_HIP(hipStreamSynchronize(s));
    }
    LOWD_HIP(hipGetLastError());
    LOWD_HIP(hipStreamSynchronize(s));
    res.n_h = (int32_t)N;
    res.m_h = M;
    return res;
}

PruneResult run_prune(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                      uint8_t *node_keep, int32_t *relabel, int32_t *h_src, int32_t *h_dst,
                      int64_t *edge_map, hipStream_t s) {
    const size_t need = prune_ws_bytes(n, m, h_src != nullptr, edge_map != nullptr);
    DBuf<char> buf(need);
    Arena ws(buf.p, buf.bytes());
    return run_prune_ws(n, m, src, dst, node_keep, relabel, h_src, h_dst, edge_map, ws, s);
}

size_t prune_ws_bytes(int32_t n, int64_t m, bool h_edges, bool edge_map) {
    Arena measure;
    int32_t dummy_out = 0;
    int64_t dummy_map = 0;
    run_prune_ws(n, m, nullptr, nullptr, nullptr, nullptr, h_edges ? &dummy_out : nullptr,
                 h_edges ? &dummy_out : nullptr, edge_map ? &dummy_map : nullptr, measure,
                 nullptr);
    return measure.peak;
}

// total = (lo, hi) of the sum of k 128-bit degrees, in two passes
static void sum_degrees(int64_t k, const uint64_t *dlo, const uint64_t *dhi, uint64_t *part_lo,
                        uint64_t *part_hi, uint64_t *total, hipStream_t s) {
    const int32_t nb = (int32_t)grid_for(k, kSumBlock, 1024);
    hipLaunchKernelGGL(k_sum_u128, dim3((unsigned)nb), dim3(kSumBlock), 0, s, k, dlo, dhi, part_lo,
                       part_hi);
    hipLaunchKernelGGL(k_sum_u128, dim3(1), dim3(kSumBlock), 0, s, (int64_t)nb, part_lo, part_hi,
                       total, total + 1);
}

PruneResult run_prune_weighted(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                               const float *w, uint8_t *node_keep, int32_t *relabel,
                               int32_t *h_src, int32_t *h_dst, float *h_w, int64_t *edge_map,
                               double *w_h, hipStream_t s) {
    PruneResult res;
    const unsigned gn = grid_for(n, 256);
    Csr csr;
    build_incidence(n, m, src, dst, csr, s);
    DBuf<int32_t> stamp((size_t)n), list_a((size_t)n), list_b((size_t)n), removed((size_t)n),
        range(2);
    DBuf<uint64_t> wi((size_t)(m > 0 ? m : 1)), dlo((size_t)n), dhi((size_t)n), part_lo(1024),
        part_hi(1024), total(2);
    DBuf<int64_t> f_rm((size_t)n), f_keep((size_t)n), p_rm((size_t)n), p_keep((size_t)n), tot(2);
    int64_t big = n > m ? (int64_t)n : m;
    DBuf<char> scan_tmp(exclusive_scan_tmp_bytes(big));
    LOWD_HIP(hipMemsetAsync(stamp.p, 0, (size_t)n * sizeof(int32_t), s));
    int32_t qmin = 0;
    fixed_point_weights(m, w, wi.p, &qmin, range.p, s);
    hipLaunchKernelGGL(k_iota, dim3(gn), dim3(256), 0, s, n, list_a.p);
    int32_t *alive = list_a.p;
    int64_t nalive = n;
    for (int32_t round = 1; nalive > 0 && m > 0; ++round) {
        hipLaunchKernelGGL(k_weighted_degrees, dim3(grid_for(nalive * kWave, 256)), dim3(256), 0,
                           s, nalive, alive, csr.row_ptr.p, csr.inc.p, src, dst, stamp.p, wi.p,
                           dlo.p, dhi.p);
        sum_degrees(nalive, dlo.p, dhi.p, part_lo.p, part_hi.p, total.p, s);
        const unsigned gc = grid_for(nalive, 256);
        hipLaunchKernelGGL(k_weighted_test, dim3(gc), dim3(256), 0, s, nalive, dlo.p, dhi.p,
                           nalive, total.p, total.p + 1, f_rm.p, f_keep.p);
        exclusive_scan_i64(f_rm.p, p_rm.p, nalive, tot.p, scan_tmp.p, scan_tmp.bytes(), s);
        exclusive_scan_i64(f_keep.p, p_keep.p, nalive, tot.p + 1, scan_tmp.p, scan_tmp.bytes(), s);
        int32_t *out = (alive == list_a.p) ? list_b.p : list_a.p;
        hipLaunchKernelGGL(k_split, dim3(gc), dim3(256), 0, s, nalive, alive, f_rm.p, p_rm.p,
                           p_keep.p, removed.p, out);
        int64_t t[2];
        LOWD_HIP(hipMemcpyAsync(t, tot.p, sizeof(t), hipMemcpyDeviceToHost, s));
        LOWD_HIP(hipStreamSynchronize(s));
        if (t[0] == 0) break;
        hipLaunchKernelGGL(k_stamp, dim3(grid_for(t[0], 256)), dim3(256), 0, s, t[0], removed.p,
                           stamp.p, round);
        alive = out;
        nalive = t[1];
        res.rounds = round;
    }
    // outputs: mask, renumbering, compacted edge list with weights
    hipLaunchKernelGGL(k_keep_flags, dim3(gn), dim3(256), 0, s, n, stamp.p, node_keep, f_keep.p);
    exclusive_scan_i64(f_keep.p, p_keep.p, n, tot.p, scan_tmp.p, scan_tmp.bytes(), s);
    if (relabel)
        hipLaunchKernelGGL(k_relabel, dim3(gn), dim3(256), 0, s, n, f_keep.p, p_keep.p, relabel);
    int64_t mh = 0;
    if (m > 0) {
        const int64_t nt = compact_tiles(m);
        DBuf<uint8_t> ekeep((size_t)m);
        DBuf<int64_t> tcount((size_t)nt), toff((size_t)nt), etot(1);
        compact_edges(m, src, dst, w, stamp.p, nullptr, p_keep.p, h_src, h_dst, h_w, edge_map,
                      ekeep.p, tcount.p, toff.p, etot.p, scan_tmp.p, scan_tmp.bytes(), s);
        LOWD_HIP(hipMemcpyAsync(&mh, etot.p, sizeof(mh), hipMemcpyDeviceToHost, s));
        LOWD_HIP(hipStreamSynchronize(s));
    }
    int64_t nh = 0;
    LOWD_HIP(hipMemcpyAsync(&nh, tot.p, sizeof(nh), hipMemcpyDeviceToHost, s));
    LOWD_HIP(hipStreamSynchronize(s));
    if (w_h) {
        // w(E(H)) = (sum of the kept degrees) / 2, times 2^q_min, rounded once
        double v = 0.0;
        if (m > 0 && nalive > 0) {
            hipLaunchKernelGGL(k_weighted_degrees, dim3(grid_for(nalive * kWave, 256)), dim3(256),
                               0, s, nalive, alive, csr.row_ptr.p, csr.inc.p, src, dst, stamp.p,
                               wi.p, dlo.p, dhi.p);
            sum_degrees(nalive, dlo.p, dhi.p, part_lo.p, part_hi.p, total.p, s);
            uint64_t tw[2];
            LOWD_HIP(hipMemcpyAsync(tw, total.p, sizeof(tw), hipMemcpyDeviceToHost, s));
            LOWD_HIP(hipStreamSynchronize(s));
            const u128 W2 = ((u128)tw[1] << 64) | tw[0];
            v = ldexp((double)(W2 >> 1), qmin);
        }
        *w_h = v;
    }
    LOWD_HIP(hipGetLastError());
    res.n_h = (int32_t)nh;
    res.m_h = mh;
    return res;
}

}  // namespace lowd
