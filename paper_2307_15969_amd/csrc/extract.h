// extract.h -- densest-set extraction (k_extract.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lowd_internal.h"

namespace lowd {

struct ExtractArgs {
    int32_t n = 0;
    int64_t m = 0;
    bool weighted = false;
    const double *L64 = nullptr;      // [n] FP64 loads
    const int64_t *row_ptr = nullptr; // incidence CSR
    const uint32_t *inc = nullptr;
    const int32_t *src = nullptr;     // [m] edge list
    const int32_t *dst = nullptr;
    const float *w = nullptr;         // [m] or nullptr
    const uint64_t *wi = nullptr;     // [m] weighted: w / 2^wq as exact integers
    const uint64_t *wi_inc = nullptr; // [2m] weighted: wi of each incidence entry's edge
    int32_t wq = 0;
    // optional: the other end of each incidence entry and the nodes of
    // degree >= kBigRow (counted a workgroup each)
    const int32_t *adj = nullptr;     // [2m]
    const int32_t *big = nullptr;     // [nbig]
    int32_t nbig = 0;
    uint8_t *in_set = nullptr;        // [n] out
};


struct ExtractScratch {
    int64_t cap = -1;
    DBuf<uint64_t> keys, keys_alt;
    DBuf<uint32_t> vals, vals_alt;
    DBuf<int32_t> pos;
    DBuf<int64_t> hist, rev, W;   // int64 or (reinterpreted) FP64
    DBuf<int64_t> part, best;     // best[0] = index, best[1] = W at that index
    DBuf<char> tmp;
    void ensure(int64_t n);
};

// Enqueues the extraction; after the stream completes, best.p[0] holds the
// number of removed nodes i* and best.p[1] holds W(S_{i*}) (int64 for
// unweighted graphs; weighted: best.p[1..2] hold W(S_{i*}) / 2^wq as an
// exact 128-bit integer).
void launch_extract(const ExtractArgs &a, ExtractScratch &sc, hipStream_t s);

// Locally-dense decomposition read from the loads: the extraction, then the
// upper concave hull of the induced weights of the top-k prefixes of the
// descending load order.  Synchronises the stream.
struct LddScratch {
    int64_t cap_points = -1, cap_chunks = -1;
    DBuf<int64_t> ck, qk, hk, cnt, off, nv;
    DBuf<int64_t> cf, qf, hf;   // int64 or (reinterpreted) FP64
    DBuf<char> tmp;
    int64_t host_q = 0;
    void ensure(int64_t points, int64_t chunks);
};
void launch_ldd(const ExtractArgs &a, ExtractScratch &sc, LddScratch &ls, int32_t *level,
                int64_t *k_end, double *f_end, int64_t *nlevels, hipStream_t s);

// Extraction for many unweighted graphs whose nodes and edges are
// concatenated (global node ids), over the A graphs act[0..A) (the graphs
// still iterating; a retired graph's results do not change); enqueued on the
// stream, scratch owned by the caller.
struct BatchExtractScratch {
    int64_t cap_n = -1;
    int32_t cap_g = -1;
    DBuf<uint64_t> k0, k1;
    DBuf<uint32_t> v0, v1, g0, g1;
    DBuf<int32_t> pos;
    DBuf<int64_t> hist, rev, W, best;
    DBuf<char> tmp;
    void ensure(int64_t N, int32_t G);
};
struct BatchExtractArgs {
    int32_t G = 0;
    int64_t N = 0;                     // total nodes
    int64_t M = 0;                     // total edges
    const int64_t *node_ptr = nullptr; // [G+1] device
    const int64_t *edge_ptr = nullptr; // [G+1] device: graph g's edges, in graph order
    int64_t max_nodes = 0;             // nodes of the largest graph
    const int32_t *node_graph = nullptr; // [N] graph of each node
    const int32_t *gsrc = nullptr;     // [M] global node ids
    const int32_t *gdst = nullptr;
    const double *L64 = nullptr;       // [N]
    int32_t A = 0;                     // graphs extracted
    const int32_t *act = nullptr;      // [A] device: their ids
    const int64_t *seg = nullptr;      // [A+1] device: compact node offsets (prefix of sizes)
    const int32_t *rank = nullptr;     // [G] device: index in act, or -1
    int64_t Na = 0;                    // seg[A]
    uint8_t *in_set = nullptr;         // [N] out (the listed graphs' nodes)
    int64_t *num = nullptr;            // [G] out (the listed graphs)
    int64_t *den = nullptr;            // [G] out
    double *D = nullptr;               // [G] out: largest load per graph
};
void launch_extract_batch(const BatchExtractArgs &a, BatchExtractScratch &sc, hipStream_t s);

// wi_inc[j] = wi[edge of incidence entry j] for the 2m entries, so that the
// weighted extraction reads each row's weights in row order instead of
// gathering them by edge
void build_entry_weights(int64_t m, const uint32_t *inc, const uint64_t *wi, uint64_t *wi_inc,
                         hipStream_t s);

}  // namespace lowd
