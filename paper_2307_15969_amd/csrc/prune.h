// prune.h -- Algorithm 2 (Pruning) on the GPU (k_prune.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lowd_internal.h"

namespace lowd {

struct PruneResult {
    int32_t rounds = 0;
    int32_t n_h = 0;
    int64_t m_h = 0;
};

// Inputs validated by the caller.  Outputs as documented for lowd_prune.
PruneResult run_prune(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                      uint8_t *node_keep, int32_t *relabel, int32_t *h_src, int32_t *h_dst,
                      int64_t *edge_map, hipStream_t s);

// The same, every device buffer taken from `ws` (nothing allocated);
// prune_ws_bytes gives the bytes it takes (h_edges: H's edge list is
// written; edge_map: the edge map is written).
PruneResult run_prune_ws(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                         uint8_t *node_keep, int32_t *relabel, int32_t *h_src, int32_t *h_dst,
                         int64_t *edge_map, Arena &ws, hipStream_t s);
size_t prune_ws_bytes(int32_t n, int64_t m, bool h_edges, bool edge_map);

// Algorithm 2 on a weighted graph, deciding every removal exactly (see
// k_prune.hip); h_w receives the kept edges' weights, w_h the kept graph's
// total weight (rounded once to FP64).
PruneResult run_prune_weighted(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                               const float *w, uint8_t *node_keep, int32_t *relabel,
                               int32_t *h_src, int32_t *h_dst, float *h_w, int64_t *edge_map,
                               double *w_h, hipStream_t s);

// Greedy peeling (Algorithm 3) of an unweighted graph, exactly: the removal
// order, |E(S)| after each removal, and S* (in_set, may be nullptr); returns
// the number of removals before S*.  Fails (LOWD_E_UNSUPPORTED) when the
// bucket bitsets would exceed max_bytes.
int64_t greedy_peel(int32_t n, int64_t m, const int32_t *src, const int32_t *dst, int32_t *order,
                    int64_t *rem_m, uint8_t *in_set, int64_t max_bytes, hipStream_t s);

}  // namespace lowd
