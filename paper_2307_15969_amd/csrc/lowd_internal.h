// lowd_internal.h -- shared declarations between the host orchestration
// (api.hip, schedule.cpp) and the device kernels (k_*.hip).  Not installed.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/lowd.h"

namespace lowd {

// ---------------------------------------------------------------- errors --
struct Error {
    int32_t status;
    std::string msg;
};
[[noreturn]] void fail(int32_t status, const std::string &msg);
void hip_check(hipError_t e, const char *what);
#define LOWD_HIP(call) ::lowd::hip_check((call), #call)

// Owning device buffer (hipMalloc / hipFree).
template <class T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    DBuf() = default;
    explicit DBuf(size_t count) { alloc(count); }
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    DBuf(DBuf &&o) noexcept : p(o.p), n(o.n) { o.p = nullptr; o.n = 0; }
    DBuf &operator=(DBuf &&o) noexcept {
        if (this != &o) { release(); p = o.p; n = o.n; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DBuf() { release(); }
    void alloc(size_t count) {
        release();
        if (count == 0) count = 1;
        LOWD_HIP(hipMalloc((void **)&p, count * sizeof(T)));
        n = count;
    }
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
    size_t bytes() const { return n * sizeof(T); }
};

// Carves device buffers out of one region, 256-byte aligned, in the order
// they are taken.  A region without a base only measures (every take returns
// nullptr): the same sequence of takes then gives the bytes a call needs.
// mark()/release(mark) give back everything taken after the mark.
struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0, peak = 0;
    Arena() = default;
    Arena(void *b, size_t c) : base((char *)b), cap(c) {}
    template <class T>
    T *take(size_t count) {
        used = (used + 255) & ~(size_t)255;
        T *p = base ? reinterpret_cast<T *>(base + used) : nullptr;
        used += (count > 0 ? count : 1) * sizeof(T);
        if (used > peak) peak = used;
        if (base && used > cap) fail(LOWD_E_UNSUPPORTED, "workspace too small");
        return p;
    }
    size_t mark() const { return used; }
    void release(size_t m) { used = m; }
};

// Slot encoding of a star leaf: bits 0..30 node id (global or LDS-local),
// bit 31 set when the star's center is the edge's dst (so the leaf is src).
// Padding slots name the infinite dummy node (n + 1, or the tail's second
// dummy) with orientation bit 0.
constexpr uint32_t kCenterIsDst = 0x80000000u;
constexpr int kWave = 64;
// "no next station" (padding slots, lanes without a star); station entries
// stay below it
constexpr uint32_t kNoStation = 0x7FFFFFFFu;
// Whole-GPU phases of at least this many edges are pulled (Schedule::pull);
// narrower ones, where the extra dependent round trip costs more than the
// scattered writes, are pushed (pulling every phase of 64K edges or more
// made a 64M-edge Chung-Lu sweep 4% slower, and its phases of 1M to 2M
// edges lost a little too; uniform 2.2M-edge phases gain 7%).
constexpr int64_t kPullMinEdges = (int64_t)1 << 21;

// ------------------------------------------------------------- schedule --
// Stars of a phase are sorted by size (descending) and dealt to tiles of 64,
// one star per lane, so tile depths are non-increasing.  T[k] = number of
// tiles of the phase deeper than k; tile t is depth_t = #{k : T[k] > t} rows
// deep and its rows are contiguous:
//   slot(t, k, lane) = slot_base + 64 * (sum_k' min(T[k'], t)) + 64 * k + lane
// (the tiles before t hold sum_{i<t} depth_i = sum_k' min(T[k'], t) rows).
// Every slot address follows from the phase descriptor alone (a kernel
// argument), so a phase needs no metadata load before its slot rows.
constexpr int kMaxStar = 32;          // largest star of a schedule (whole-GPU phases)
constexpr int kTierStar = 16;         // largest star of the single-workgroup tiers and batches
constexpr int kTailWaves = 8;         // waves of the LDS-resident tail workgroup

template <int D>
struct PhaseDescT {
    static constexpr int kDepth = D;
    int64_t slot_base;                // first slot of the phase
    int32_t tile0;                    // first tile (index into tile_center / 64)
    int32_t T[D];                     // T[k] = tiles of depth > k; T[0] = tiles
    int32_t sink;                     // entry that takes the stores of stations without a
                                      // next one (the last entry; unused by the LDS tiers)
};
// the schedule's descriptors and the whole-GPU phase kernels
using PhaseDescWide = PhaseDescT<kMaxStar>;
// the single-workgroup tiers and the batches, which stage descriptors in LDS
// and take tiles of at most kTierStar rows
using PhaseDesc = PhaseDescT<kTierStar>;

// A descriptor in the narrower form (its phase is at most D rows deep).
template <int D, int E>
inline PhaseDescT<D> narrow_desc(const PhaseDescT<E> &w) {
    PhaseDescT<D> d;
    d.slot_base = w.slot_base;
    d.tile0 = w.tile0;
    for (int k = 0; k < D; ++k) d.T[k] = w.T[k];
    d.sink = w.sink;
    return d;
}
// rows of the phase's deepest tile
template <int D>
inline int32_t desc_depth(const PhaseDescT<D> &d) {
    int32_t k = 0;
    while (k < D && d.T[k] > 0) ++k;
    return k;
}

// LDS bytes the tail workgroup spends on its phase descriptors.
__host__ __device__ inline size_t tail_desc_bytes(int64_t nph) {
    return ((size_t)nph * sizeof(PhaseDesc) + 15) & ~(size_t)15;
}

// Host-side result of the phase schedule and its device layout.
struct Schedule {
    int32_t n = 0;
    int64_t m = 0;
    int32_t smax = 16;
    int32_t P = 0;                  // phases
    std::vector<int32_t> phase;     // per edge
    std::vector<int32_t> center;    // per edge (node id)
    int32_t P1 = 0;                 // phases [0, P1) run as whole-GPU launches
    int32_t P0 = 0;                 // [P1, P0) in one workgroup, loads in global memory;
                                    // [P0, P) in one workgroup, loads in LDS
    std::vector<PhaseDescWide> desc;      // [P]
    std::vector<int32_t> tile_center;     // [ntiles*64] node id (local ids for tail tiles), -1 empty
    std::vector<uint32_t> slot_leaf;      // [nslots] leaf | orientation (padding: dummy leaf)
    std::vector<int64_t> slot_edge;       // [nslots] edge index, -1 for padding
    std::vector<int64_t> edge_slot;       // [m] slot of each edge
    std::vector<int32_t> tail_nodes;      // global ids of the nodes held in LDS by the tail
    int64_t tail_edges = 0;
    // Station layout of the node loads.  A node's load is kept at the place
    // where the sweep uses it next: one entry per leaf slot and per tile
    // lane of the phases before P0 (the slot's or the lane's own index, the
    // lanes after the slots), one per node of the tail, and a home entry
    // for nodes on no edge.  Each station names its node's next station in
    // sweep order (the last one names the first), so a phase reads its loads
    // in slot order and writes each updated load to where it is read next.
    int64_t center_base = 0;              // entry of tile lane i: center_base + i
    int64_t tail_base = 0;                // entry of tail node j: tail_base + j
    int64_t entries = 0;                  // size of the entry array
    std::vector<uint32_t> slot_next;      // [nslots] next station | orientation bit; padding: kNoStation
    std::vector<uint32_t> center_next;    // [ntiles*64] next station of the lane's center; empty: kNoStation
    std::vector<uint32_t> tail_next;      // [ntail] station after the tail (the node's first)
    std::vector<uint32_t> home;           // [n] where each node's load rests between sweeps
    // Pulled phases (empty when none): their stations read each node's load
    // from its previous station, which keeps its own output.
    std::vector<uint8_t> pull;            // [P] 1 for a pulled whole-GPU phase
    std::vector<uint32_t> slot_src;       // [nslots] entry a pulled slot reads
    std::vector<uint32_t> center_src;     // [ntiles*64] entry a pulled lane's center reads
    std::vector<int64_t> phase_edges;     // [P]
    std::vector<int32_t> phase_depth;     // [P] deepest star
};

// Builds the phase schedule (first fit over the edges in visiting order) and
// the tile layout.
// lds_bytes bounds the single-workgroup tiers' LDS (descriptors, and node
// loads of l_bytes each for the last tier; 0 = whole-GPU launches only);
// force_p0 / force_p1 >= 0 ask for the splits (P0 moved later until the tail
// fits; P1 clamped to P0); force_p0 == -2 computes the phase assignment only.
// whole_in_lds: every phase runs from LDS with node ids unchanged (all n
// nodes staged; dummies n and n + 1) -- the batched form; the caller checks
// that the graph fits.  pull_min_edges >= 0: whole-GPU phases of at least
// that many edges are pulled (Schedule::pull); -1: none.
void build_schedule(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, int32_t smax,
                    int64_t lds_bytes, int64_t l_bytes, int64_t force_p0, int64_t force_p1,
                    Schedule &out, bool whole_in_lds = false, int64_t pull_min_edges = -1);

// --------------------------------------------------------------- kernels --
typedef unsigned __int128 u128;

// Device-wide primitives (k_scan.hip)
void exclusive_scan_i64(const int64_t *in, int64_t *out, int64_t n, int64_t *total_dev,
                        void *tmp, size_t tmp_bytes, hipStream_t s);
void exclusive_scan_f64(const double *in, double *out, int64_t n, double *total_dev, void *tmp,
                        size_t tmp_bytes, hipStream_t s);
void exclusive_scan_u128(const u128 *in, u128 *out, int64_t n, u128 *total_dev, void *tmp,
                         size_t tmp_bytes, hipStream_t s);
size_t exclusive_scan_tmp_bytes(int64_t n);

// Weights as exact integers (k_prune.hip): every float32 weight is M * 2^E
// with an integer M < 2^24 (E its ulp exponent); with q the smallest E over
// the edges, wi[e] = w[e] / 2^q is an integer, below 2^64 when the
// exponents span at most 40 binades (else LOWD_E_UNSUPPORTED).  range_dev:
// 2 ints of device scratch.  Synchronises the stream.
constexpr int32_t kMaxExpSpan = 40;
void fixed_point_weights(int64_t m, const float *w, uint64_t *wi, int32_t *q_out,
                         int32_t *range_dev, hipStream_t s);

// One count of digit d in the LDS counters h, for every active lane: the
// lanes whose digit equals the first active lane's add theirs with one
// atomic.  Sorted or clustered keys (a node's incidence entries, a pass's
// input after the previous pass) put whole waves on one counter, and the
// LDS serialises atomics to one address: on 520M keys of runs a histogram
// pass took 1.7 ms against 0.5 ms for random keys, and 0.5 ms counted so.
__device__ inline void count_digit(uint32_t *h, uint32_t d) {
    const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
    const uint64_t same = __ballot(d == d0);
    if (d == d0) {
        if ((uint32_t)__lane_id() == (uint32_t)(__ffsll((unsigned long long)same) - 1))
            atomicAdd(&h[d0], (uint32_t)__popcll(same));
    } else {
        atomicAdd(&h[d], 1u);
    }
}

// x rounded once to FP64 (round to nearest even), on either side
__host__ __device__ inline double u128_to_double(u128 x) {
    const uint64_t hi = (uint64_t)(x >> 64);
    if (hi == 0) return (double)(uint64_t)x;
    // keep the top 64 bits and fold every lower bit into a sticky bit, so the
    // one rounding of the 64-bit value is the rounding of x
    int shift = 64;
    uint64_t h = hi;
    while (h) {
        h >>= 1;
        --shift;
    }
    shift = 64 - shift;   // bits of hi
    const uint64_t top = (uint64_t)(x >> shift);
    const bool sticky = (x & ((((u128)1) << shift) - 1)) != 0;
    double r = (double)(top | (sticky ? 1u : 0u));
    for (int k = 0; k < shift; ++k) r *= 2.0;
    return r;
}
// Stable LSD radix sort of (key, value) pairs on bits [0, bits) of the key;
// vals and vals_alt may both be NULL to sort the keys alone.
void radix_sort_u32(uint32_t *keys, uint32_t *vals, uint32_t *keys_alt, uint32_t *vals_alt,
                    int64_t n, int bits, void *tmp, size_t tmp_bytes, bool *result_in_alt,
                    hipStream_t s);
void radix_sort_u64(uint64_t *keys, uint32_t *vals, uint64_t *keys_alt, uint32_t *vals_alt,
                    int64_t n, int bits, void *tmp, size_t tmp_bytes, bool *result_in_alt,
                    hipStream_t s);
size_t radix_sort_tmp_bytes(int64_t n);
// One stable pass of that sort over keys alone, on the digit
// (key >> shift) & 255: keys_out holds the keys grouped by digit, starts
// (device, 257 entries) the first position of each digit and n at the end.
// tmp: radix_sort_tmp_bytes(n).
void radix_partition_u32(const uint32_t *keys, uint32_t *keys_out, int64_t n, int shift,
                         int64_t *starts, void *tmp, size_t tmp_bytes, hipStream_t s);

// Graph validation (k_graph.hip): first bad edge index or -1 in *bad_dev.
void launch_validate(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                     const float *w, int64_t *bad_dev, hipStream_t s);
// Index of the later edge of the first repeated unordered pair, or -1.
int64_t find_duplicate_pair(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                            hipStream_t s);
// The same with its sort buffers taken from `ws` (released again on return);
// with `invalid` it also checks the edges as launch_validate does (w: the
// weights or NULL), *invalid = the first invalid edge or -1, and looks for
// a repeat only when there is none.
int64_t find_duplicate_pair_ws(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                               Arena &ws, hipStream_t s, const float *w = nullptr,
                               int64_t *invalid = nullptr);
// Incidence CSR, rows in ascending edge index: entry j = 2*e + side
// (side 0: the row node is src[e]; side 1: dst[e]).  row_ptr has n+1 entries.
// Rows (incidence rows, i.e. node degrees) of at least this length are
// handled by a wave or a workgroup each in the per-node kernels; shorter rows
// by one thread or a group of 8 lanes.
constexpr int32_t kBigRow = 256;

struct Csr {
    DBuf<int64_t> row_ptr;   // [n+1]
    DBuf<uint32_t> inc;      // [2m]
};
void build_incidence(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, Csr &csr,
                     hipStream_t s);
// adj[j] = the other end of the edge of incidence entry j ([2m])
void build_adjacency(int64_t m, const Csr &csr, const int32_t *src, const int32_t *dst,
                     int32_t *adj, hipStream_t s);
inline unsigned grid_for(int64_t work, int block, int64_t cap = 65536) {
    int64_t g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

}  // namespace lowd
