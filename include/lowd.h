/*
 * lowd.h -- C interface of liblowd.so, the MI355X (gfx950) implementation of
 * the LOWD densest-subgraph method: Locally Optimal Weight Distribution
 * (Algorithm 1) and its pruning pre-process (Algorithm 2) from Zhu, Liu, Feng,
 * Cheng, "Fast Searching The Densest Subgraph And Decomposition With Local
 * Optimality" (arXiv 2307.15969).  Besides the solver: the locally-dense
 * decomposition read-out (Problem 2) and Corollary 1's bounds, convergence
 * traces, greedy peeling (the appendix's Algorithm 3) as Algorithm 2's
 * plug-in solver, and a batched form for many small graphs.
 *
 * Conventions for every entry point
 *  - Graphs are COO edge lists, one entry per undirected edge (Section II,
 *    Problem 1: G = (V, E, W), w_e > 0, w_e = 1 when unweighted).  Node ids
 *    are int32 in [0, n); an edge list must be simple: src[e] != dst[e], no
 *    unordered pair twice.  Weights are float32 > 0 and finite, or NULL for
 *    an unweighted graph.
 *  - Pointers marked [device] are HIP device pointers that the caller owns;
 *    the library borrows them for the duration of the call (or, for a
 *    solver, until lowd_solver_free) and never frees them.  Pointers marked
 *    [host] are ordinary host memory.
 *  - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *    Work is enqueued on that stream.  Calls that return host values
 *    synchronise the stream before returning; that is stated per call.
 *  - Every call returns a lowd_status.  Negative values are errors; the
 *    message of the last error on the calling thread is available from
 *    lowd_last_error().  No C++ exception crosses this interface.
 */
#ifndef LOWD_H
#define LOWD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t lowd_status;
#define LOWD_OK 0
#define LOWD_NOT_CONVERGED 1    /* informational: the sweep limit came before the tolerance */
#define LOWD_E_ARG (-1)         /* bad pointer, size or option */
#define LOWD_E_GRAPH (-2)       /* id out of range, self-loop, repeated pair, bad weight */
#define LOWD_E_HIP (-4)         /* a HIP runtime call failed */
#define LOWD_E_UNSUPPORTED (-5) /* valid request beyond a documented limit (e.g. a batch graph larger than one workgroup's LDS) */
#define LOWD_E_NOMEM (-6)       /* host or device allocation failed */

/* Precision of the solver state (edge fractions and node loads). */
#define LOWD_STATE_F64 0  /* FP64 fractions and loads; bit-reproducible */
#define LOWD_STATE_F32K 1 /* FP32 fractions, FP32 loads with a compensation term */

typedef struct lowd_solver lowd_solver;

/* Library version string. */
const char *lowd_version(void);

/* Message of the last failed call on this thread ("" if none).  Valid until
 * the next call on the same thread. */
const char *lowd_last_error(void);

/*
 * lowd_prune -- Algorithm 2 (Pruning) on an unweighted graph, with the
 * counting-sort bucket scheme of Section III-D: starting from H = G, each
 * round removes every node whose degree in H is below the density
 * rho(H) = |E(H)| / |V(H)| (decided exactly as deg * |V(H)| < |E(H)|), then
 * recomputes rho(H); it stops when a round removes nothing.  By the degree
 * bound of Theorem 4 no node of a densest subgraph is removed.
 *
 *   n, m          nodes and edges of G (n >= 1, m >= 0)
 *   src, dst      [device] int32[m] edge list of G
 *   node_keep     [device] uint8[n] out: 1 if the node is in H
 *   relabel       [device] int32[n] out: id of the node in H (kept nodes are
 *                 numbered 0..n_h-1 in ascending original id), -1 if removed;
 *                 may be NULL
 *   h_src, h_dst  [device] int32[m] out: the edge list of H in H's ids, the
 *                 kept edges in their original relative order (the first
 *                 *m_h entries are written); may both be NULL
 *   edge_map      [device] int64[m] out: original index of each H edge; may
 *                 be NULL
 *   rounds, n_h, m_h  [host] out: removal rounds, |V(H)|, |E(H)|
 * Synchronises `stream`.  Weighted graphs: lowd_prune_weighted.
 */
lowd_status lowd_prune(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                       uint8_t *node_keep, int32_t *relabel, int32_t *h_src, int32_t *h_dst,
                       int64_t *edge_map, int32_t *rounds, int32_t *n_h, int64_t *m_h,
                       void *stream);

/*
 * lowd_prune_noalloc -- lowd_prune for callers that cannot allocate device
 * memory (tight serving loops, harnesses that forbid hipMalloc): the same
 * arguments, the same results bit for bit, but every device buffer of the
 * validation and the prune (edge lists, degree buckets, radix pass and
 * scan scratch) comes from one file-scope device array of 128 MiB that each GPU
 * holds from the library's load until the process ends; the call makes no
 * hipMalloc, hipFree or other allocating call.  A graph whose buffers would
 * exceed 128 MiB (about 29 bytes per edge plus 56 per node) is rejected
 * with LOWD_E_UNSUPPORTED before any device work.  Every call on one GPU
 * uses that GPU's one array and keeps what the last call left there, so
 * calls that overlap on one GPU (other threads, other streams) race: the
 * caller serialises them.  Buffers that must start at zero are cleared by
 * the call itself.  Synchronises `stream`.
 */
lowd_status lowd_prune_noalloc(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                               uint8_t *node_keep, int32_t *relabel, int32_t *h_src,
                               int32_t *h_dst, int64_t *edge_map, int32_t *rounds, int32_t *n_h,
                               int64_t *m_h, void *stream);

/*
 * lowd_prune_weighted -- Algorithm 2 on a weighted graph (Section III-D: each
 * round scans the nodes still in H): every round removes each node whose
 * weighted degree in H is below rho(H) = w(E(H)) / |V(H)|, until a round
 * removes nothing.  The test is exact: the float32 weights are integer
 * multiples of 2^q for the smallest q among them, so degrees and w(E(H))
 * are summed exactly in 128-bit integers and compared exactly (weights
 * whose binary exponents span more than 40 give LOWD_E_UNSUPPORTED).
 *
 *   w      [device] float32[m] positive finite weights of G
 *   h_w    [device] float32[m] out: weights of H's edges (first *m_h); may
 *          be NULL
 *   w_h    [host] out: w(E(H)) rounded once to FP64; may be NULL
 *   other arguments as for lowd_prune
 * Synchronises `stream`.
 */
lowd_status lowd_prune_weighted(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                                const float *w, uint8_t *node_keep, int32_t *relabel,
                                int32_t *h_src, int32_t *h_dst, float *h_w, int64_t *edge_map,
                                int32_t *rounds, int32_t *n_h, int64_t *m_h, double *w_h,
                                void *stream);

/*
 * lowd_greedy_peel -- greedy peeling (the appendix's Algorithm 3), the second
 * solver Algorithm 2's pruning can feed: from S = V and S* = V, repeatedly
 * remove a node of minimum degree in S (ties: the smallest id) with its
 * edges, replacing S* by S whenever rho(S) > rho(S*).  Exactly the
 * sequential definition; one workgroup runs the removals over bucket
 * bitsets in device memory ((largest degree + 1) * n / 8 bytes: graphs that
 * would need more than 32 GiB give LOWD_E_UNSUPPORTED -- prune them first).
 * By Theorem 5 the first n - n_h removals are exactly the nodes lowd_prune
 * removes, so greedy on the pruned graph continues greedy on G.
 *   order   [device] int32[n] out: removal order
 *   rem_m   [device] int64[n] out: |E(S)| after each removal
 *   in_set  [device] uint8[n] out: S*; may be NULL
 *   num, den [host] out: |E(S*)|, |S*|; may be NULL
 * Unweighted graphs.  Synchronises `stream`.
 */
lowd_status lowd_greedy_peel(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                             int32_t *order, int64_t *rem_m, uint8_t *in_set, int64_t *num,
                             int64_t *den, void *stream);

/*
 * lowd_init_loads -- Algorithm 1, initialisation: every edge gives half its
 * weight to each endpoint (f_e(u) = f_e(v) = w_e / 2) and the load of a node
 * is the sum of the halves it receives, summed in ascending edge index.
 * Also validates the graph and builds, once, the edge schedule the sweeps
 * follow: the edges are split into phases, each phase a set of vertex-
 * disjoint stars of at most `star_max` leaves (the center of an edge is its
 * endpoint of larger degree, ties to the smaller id; the edges are visited in
 * ascending order of the e-th output of SplitMix64 seeded with 0, ties by
 * index, and edge e joins the first phase where its center is not a leaf and
 * has fewer than star_max leaves and its leaf is unused).  A sweep processes
 * the phases in order; the result equals processing the edges one by one in
 * ascending (phase, edge index).
 *
 * How a sweep runs (none of this changes the result): the wide phases as one
 * launch each, the next narrower ones inside one workgroup with the loads in
 * global memory, and the last, narrowest ones inside one workgroup with
 * their nodes' loads in LDS.  A cost model places the two splits;
 * LOWD_MID_SPLIT and LOWD_TAIL_SPLIT in the environment (read by this call)
 * override them.  Between phases a node's load waits where the sweep reads
 * it next (its next leaf slot or star).  LOWD_LAYOUT=node in the
 * environment keeps the loads in one node-indexed array instead, gathered
 * and scattered by id, every phase a launch of its own (measured slower on
 * every graph tried; the results are the same bits).
 *
 *   n, m          nodes and edges (n >= 1, m >= 0, m < 2^31)
 *   src, dst      [device] int32[m]; read during this call only
 *   w             [device] float32[m] or NULL (unit weights); read during
 *                 this call only
 *   state         LOWD_STATE_F64 or LOWD_STATE_F32K
 *                 (weighted graphs whose weights' binary exponents span more
 *                 than 40 give LOWD_E_UNSUPPORTED: the extraction's exact
 *                 integer sums need them closer)
 *   star_max      leaves per star per phase, 1..32 (1 gives a proper edge
 *                 colouring: every phase is a matching); 16 is the default.
 *                 Phases whose stars have more than 16 leaves run as
 *                 whole-GPU launches only (the single-workgroup tiers take
 *                 tiles of at most 16 rows)
 *   out           [host] receives the solver; free with lowd_solver_free
 * The solver owns its device memory (schedule, fractions, loads, about
 * 40 bytes per edge and 40 per node for LOWD_STATE_F64).  Synchronises
 * `stream`.  LOWD_E_GRAPH names the first offending edge.
 */
lowd_status lowd_init_loads(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                            const float *w, int32_t state, int32_t star_max, lowd_solver **out,
                            void *stream);

/*
 * lowd_reset_loads -- returns the solver to Algorithm 1's initial state
 * (f_e = w_e / 2 on both ends, loads as after lowd_init_loads) without
 * rebuilding the schedule.  Asynchronous on `stream`.
 */
lowd_status lowd_reset_loads(lowd_solver *s, void *stream);

/*
 * lowd_iterate -- `sweeps` passes of Algorithm 1's edge loop: for each edge
 * (u, v), if l_u > l_v move d = min((l_u - l_v)/2, f_e(u)) from u to v,
 * otherwise move d = min((l_v - l_u)/2, f_e(v)) from v to u.  With
 * LOWD_STATE_F64 the result is bit-identical to the sequential loop in
 * schedule order.  Asynchronous: only enqueues work on `stream`.
 */
lowd_status lowd_iterate(lowd_solver *s, int32_t sweeps, void *stream);

/*
 * lowd_check -- convergence statistics of the current state (Section III-B):
 * D = max_u l_u, the dual objective (an upper bound on the maximum density
 * by weak duality), the sum of loads (equal to the total weight) and the QP
 * objective sum_u l_u^2 (Section III-C).  For LOWD_STATE_F32K the loads are
 * first recomputed in FP64 from the FP32 fractions, so D is the objective of
 * a feasible dual point.  Any output may be NULL.  Synchronises `stream`.
 */
lowd_status lowd_check(lowd_solver *s, double *D, double *sum_loads, double *sum_sq_loads,
                       void *stream);

/*
 * lowd_extract_densest -- Algorithm 1, extraction: sort the nodes by load,
 * ascending (stable on node id), remove them one by one and keep the
 * remaining set of largest density, the first (largest) one on ties; the
 * empty set is never a candidate.  Densities use the graph's own weights
 * (Problem 1) and are compared exactly: unweighted graphs give an exact
 * rational num_unit / den; for weighted graphs every float32 weight is an
 * exact integer multiple of the smallest weight's unit in the last place,
 * so W(S) is an exact integer sum, returned as num_w rounded once to FP64.
 * Loads are FP64 (for LOWD_STATE_F32K the FP64 recomputation from the
 * fractions).
 *
 *   in_set    [device] uint8[n] out: 1 if the node is in the extracted set
 *   num_unit  [host] out: |E(S*)| for an unweighted graph, else 0; may be NULL
 *   num_w     [host] out: W(S*) as FP64; may be NULL
 *   den       [host] out: |S*|; may be NULL
 *   D         [host] out: max load (as lowd_check); may be NULL
 *   gap       [host] out: (D - rho) / rho with rho = num / den; may be NULL
 * Synchronises `stream`.
 */
lowd_status lowd_extract_densest(lowd_solver *s, uint8_t *in_set, int64_t *num_unit,
                                 double *num_w, int64_t *den, double *D, double *gap,
                                 void *stream);

/*
 * lowd_check_kept, lowd_extract_densest_kept -- lowd_check and
 * lowd_extract_densest on the loads the solver keeps, with the same
 * arguments: for LOWD_STATE_F32K each node's compensated FP32 pair rounded
 * to FP64, without the recomputation from the fractions; for
 * LOWD_STATE_F64 identical to the plain calls.  The kept FP32K loads follow
 * the fractions' sums up to the rounding of the FP32 fractions (Section
 * III-B's bound needs the loads of the fractions as stored), so D here
 * estimates the dual objective: it steers the iteration between checks, and
 * a certificate takes D from lowd_check.  The extracted set is a set of the
 * graph, its density exact as for lowd_extract_densest.
 */
lowd_status lowd_check_kept(lowd_solver *s, double *D, double *sum_loads, double *sum_sq_loads,
                            void *stream);

/*
 * lowd_resync_loads -- LOWD_STATE_F32K: sets every node's carried
 * compensated load to the FP64 load recomputed from the stored fractions
 * (as lowd_check computes it), rounded to the (s, c) pair.  A step moves
 * the carried loads by its exact amount while the FP32 fraction takes the
 * rounded one, so over many sweeps the carried loads can drift from the
 * loads of the stored fractions, which alone make the dual bound; this
 * restarts them from those.  No-op for LOWD_STATE_F64 (its loads are the
 * loads of its fractions) and for a graph without edges.  Asynchronous.
 */
lowd_status lowd_resync_loads(lowd_solver *s, void *stream);
lowd_status lowd_extract_densest_kept(lowd_solver *s, uint8_t *in_set, int64_t *num_unit,
                                      double *num_w, int64_t *den, double *D, double *gap,
                                      void *stream);

/*
 * lowd_solve -- Algorithm 1 run to a certified density gap, from the
 * solver's current state (lowd_reset_loads first for a fresh solve).  The
 * stopping rule is Section III-B's duality: D = max load bounds the maximum
 * density from above at every sweep, and the density rho of any extracted
 * set bounds it from below, so the densest set extracted so far is
 * certified once (D - rho) / rho <= tol.  The call sweeps and checks until
 * that holds or max_sweeps sweeps are done.
 *
 * The first check comes after one sweep.  Later ones come where the decay
 * of the gap over the last two checks predicts the tolerance (at most
 * check_every sweeps on); without such a prediction the check points double,
 * but stay far enough apart that a check (timed against a sweep on the
 * stream) costs at most about a quarter of the sweeps between two checks.
 * A check takes D first and extracts (Algorithm 1's sort and prefix
 * densities) only when D does not already certify the best set.
 * With LOWD_STATE_F32K checks screen with the kept compensated loads and
 * confirm a passing gap with D recomputed in FP64 from the stored fractions
 * (the loads of a feasible dual point); when the confirmation fails the
 * carried loads restart from those loads (as lowd_resync_loads).
 *
 *   tol          relative gap to reach (>= 0; 1e-6 in the benchmarks)
 *   max_sweeps   sweep limit (>= 0)
 *   check_every  most sweeps between two checks (>= 1; 10 is the default)
 *   in_set       [device] uint8[n] out: the certified (or, on
 *                LOWD_NOT_CONVERGED, the best) set
 *   num_unit     [host] out: |E(S)| (unit weights; 0 for weighted graphs);
 *                may be NULL
 *   num_w        [host] out: W(S) in FP64; may be NULL
 *   den          [host] out: |S|; may be NULL
 *   D, gap       [host] out: the bound and the gap at the last check; may be
 *                NULL
 *   sweeps_used  [host] out: sweeps done by this call; may be NULL
 * Returns LOWD_OK when the gap is within tol, LOWD_NOT_CONVERGED (> 0, the
 * outputs still written) when max_sweeps came first, or an error.
 * Synchronises `stream`.
 */
lowd_status lowd_solve(lowd_solver *s, double tol, int32_t max_sweeps, int32_t check_every,
                       uint8_t *in_set, int64_t *num_unit, double *num_w, int64_t *den,
                       double *D, double *gap, int32_t *sweeps_used, void *stream);

/*
 * lowd_ldd_readout -- the locally-dense decomposition (Problem 2, Property
 * 2) read from the current loads: with the nodes ranked by descending load
 * (the reverse of lowd_extract_densest's order) and f(k) the weight of the
 * edges among the top k nodes, level j ends at the largest k maximising
 * (f(k) - f(k_{j-1})) / (k - k_{j-1}) (k_0 = 0), until k = n.  Level 0 is
 * the set lowd_extract_densest returns; at the limit of the iteration the
 * levels are the decomposition B_1 < B_2 < ... and lambda_j = (f_end[j] -
 * f_end[j-1]) / (k_end[j] - k_end[j-1]) its level values.  Every level end
 * is decided exactly (integer weight sums, as for lowd_extract_densest);
 * f_end is f rounded once to FP64.  Corollary 1 then bounds the
 * density of any k-node subgraph by the envelope of (k_end, f_end) at k,
 * over k.
 *   level    [device] int32[n] out: level of each node (0 = densest)
 *   k_end    [device] int64[n] out: level ends k_1 .. k_L (first L entries)
 *   f_end    [device] double[n] out: f(k_1) .. f(k_L) (exact integers for
 *            unit weights)
 *   nlevels  [host] out: L
 * Synchronises `stream`.
 */
lowd_status lowd_ldd_readout(lowd_solver *s, int32_t *level, int64_t *k_end, double *f_end,
                             int64_t *nlevels, void *stream);

/*
 * lowd_dks_bound -- Corollary 1: from a decomposition read-out, an upper
 * bound on the density of any k-node subgraph (the densest-k-subgraph and
 * at-least-k problems): the envelope (f_end[j-1] + (k - k_end[j-1]) *
 * lambda_j) / k for k_end[j-1] < k <= k_end[j].  At k = k_end[j] and the
 * limit of the iteration it is the density of B_{j+1} itself.  Host only.
 *   k_end, f_end  [host] the read-out's first nlevels entries
 *   bound         [host] out
 */
lowd_status lowd_dks_bound(const int64_t *k_end, const double *f_end, int64_t nlevels, int64_t k,
                           double *bound);

/*
 * lowd_convergence_trace -- continues the iteration for `sweeps` sweeps and
 * records, before the first and after every `every` sweeps (and at the
 * end), the quantities behind the paper's convergence curves (Section IV):
 * the dual bound D = max load (Section III-B), the density rho of the
 * extracted set, the QP objective sum of squared loads (Section III-C) and
 * the relative gap (D - rho) / rho.  The relative error (rho* - rho) / rho*
 * and the QP error sum_sq - sum_sq* follow from a reference rho*, sum_sq*
 * (for instance lambda_1 and sum_j lambda_j^2 |level j| of a converged
 * decomposition).
 *   out     [host] double[5 * (ceil(sweeps / every) + 1)] out, rows of
 *           (sweeps done, D, rho, sum_sq, gap)
 *   points  [host] out: rows written
 * Synchronises `stream` at every record.
 */
lowd_status lowd_convergence_trace(lowd_solver *s, int32_t sweeps, int32_t every, double *out,
                                   int64_t *points, void *stream);

/*
 * lowd_read_state -- copies the current fractions and loads out, in the
 * caller's edge order: x[e] = f_e(src[e]) and load[u] = l_u, both FP64
 * (LOWD_STATE_F32K: the FP32 fraction widened, and the load as its value
 * plus compensation).  Either pointer may be NULL.
 *   x     [device] double[m]
 *   load  [device] double[n]
 * Asynchronous on `stream`.
 */
lowd_status lowd_read_state(const lowd_solver *s, double *x, double *load, void *stream);

/*
 * lowd_schedule_export -- the schedule built by lowd_init_loads, per edge in
 * the caller's edge order: its phase and its star center.
 *   phase   [host] int32[m] out; may be NULL
 *   center  [host] int32[m] out; may be NULL
 *   nphases [host] out; may be NULL
 */
lowd_status lowd_schedule_export(const lowd_solver *s, int32_t *phase, int32_t *center,
                                 int32_t *nphases);

/*
 * lowd_schedule_build -- the same phase assignment as lowd_init_loads builds,
 * computed on the host from host arrays, without a GPU (for inspection and
 * for precomputing schedules); star_max may here be 1..254.
 *   src, dst  [host] int32[m], validated as for lowd_init_loads except for
 *             repeated pairs
 *   phase     [host] int32[m] out; may be NULL
 *   center    [host] int32[m] out; may be NULL
 *   nphases   [host] out; may be NULL
 */
lowd_status lowd_schedule_build(int32_t n, int64_t m, const int32_t *src, const int32_t *dst,
                                int32_t star_max, int32_t *phase, int32_t *center,
                                int32_t *nphases);

/*
 * lowd_solver_info -- sizes of the solver, for reports.
 *   info [host] int64[12] out: n, m, phases, phases run by whole-GPU
 *        launches, phases run inside one workgroup with loads in global
 *        memory, phases run inside one workgroup with loads in LDS, nodes
 *        held in LDS, edges of the LDS phases, edges of the global-memory
 *        single-workgroup phases, state type, load layout (0: stations, 1:
 *        a node-indexed array), whole-GPU phases that pull their loads
 *        (phases of at least 2^21 edges, or LOWD_PULL_EDGES: each node's
 *        load is read at its previous station, which keeps its output,
 *        instead of being written to its next one).
 */
lowd_status lowd_solver_info(const lowd_solver *s, int64_t *info);

/* Releases the solver's host and device memory (never caller memory).
 * Waits for the solver's pending work first.  NULL is accepted. */
void lowd_solver_free(lowd_solver *s);

/*
 * lowd_batch_solve -- many independent unweighted graphs, each solved to a
 * certified density gap (Section III-B, as lowd_solve), in one persistent
 * launch (captured in a HIP graph): a workgroup takes the next graph (the
 * largest first) and solves it alone, with its loads in LDS: sweeps of
 * Algorithm 1 in the graph's own schedule and, every few sweeps, a check
 * inside the workgroup: the loads' maximum D_g, then, unless D_g already
 * certifies the densest set found so far, Algorithm 1's extraction (sort by
 * load, densest removal prefix).  The graph stops at the first check where
 * (D_g - rho_g) / rho_g <= tol, rho_g the density of its densest set so
 * far, or at max_sweeps.  For LOWD_STATE_F32K the checks read the kept
 * compensated loads, and a gap within tol is confirmed with D_g recomputed
 * in FP64 from the stored fractions (the loads of a feasible dual point);
 * the carried loads then restart from those loads, so a failed
 * confirmation leaves no drift behind.
 * Checks come every check_every sweeps, sooner when the gap's decay over
 * the last two checks predicts the tolerance.  The set of each graph is
 * Algorithm 1's extraction after set_sweeps[g] sweeps of its single-graph
 * iteration (with the same star_max).
 *
 *   G            number of graphs (>= 1)
 *   node_ptr     [host] int64[G+1]: graph g owns nodes node_ptr[g]..node_ptr[g+1]-1
 *   edge_ptr     [host] int64[G+1]: graph g owns edges edge_ptr[g]..edge_ptr[g+1]-1
 *   src, dst     [device] int32[total edges], node ids local to their graph
 *   state        LOWD_STATE_F64 or LOWD_STATE_F32K
 *   star_max     as for lowd_init_loads
 *   tol          relative gap (>= 0)
 *   max_sweeps   sweep limit per graph (>= 0)
 *   check_every  most sweeps between two checks (>= 1)
 *   in_set       [device] uint8[total nodes] out
 *   num, den     [device] int64[G] out: |E(S_g)|, |S_g|
 *   D            [device] double[G] out: each graph's bound at its last check;
 *                may be NULL
 *   sweeps_used  [device] int32[G] out: sweeps each graph ran; may be NULL
 *   set_sweeps   [device] int32[G] out: the sweep count at which each
 *                graph's set was extracted; may be NULL
 * Returns LOWD_OK when every graph is within tol, LOWD_NOT_CONVERGED (> 0,
 * outputs written) when some graph reached max_sweeps first.  Every graph's
 * phase descriptors and node loads must fit one workgroup's LDS beside the
 * checks' own (about 18 KB): 80 bytes per phase plus 8 per node within
 * 160 KB - 18 KB; larger graphs give LOWD_E_UNSUPPORTED.  Synchronises
 * `stream`.
 */
lowd_status lowd_batch_solve(int32_t G, const int64_t *node_ptr, const int64_t *edge_ptr,
                             const int32_t *src, const int32_t *dst, int32_t state,
                             int32_t star_max, double tol, int32_t max_sweeps,
                             int32_t check_every, uint8_t *in_set, int64_t *num, int64_t *den,
                             double *D, int32_t *sweeps_used, int32_t *set_sweeps,
                             void *stream);

/*
 * The batched form in steps, for solving to a tolerance: a prepared batch
 * keeps its schedules, fractions and loads on the device between calls.
 * lowd_batch_solve is lowd_batch_prepare + lowd_batch_solve_prepared.
 */
typedef struct lowd_batch lowd_batch;

/*
 * lowd_batch_prepare -- validates the graphs (as lowd_batch_solve), builds
 * every graph's schedule, uploads the layout and sets Algorithm 1's initial
 * state.  With tune = 1 it also times each supported launch shape (waves
 * per workgroup, prefetching tile buffers or not, workgroups per CU) on a
 * short run of this batch and keeps the fastest; the shape never changes a
 * result.  tune = 0 keeps the default shape.  For LOWD_STATE_F32K, launches
 * made once at most two graphs per CU still iterate (as of the last
 * lowd_batch_retire) use 16 waves per workgroup, one workgroup per CU; the
 * environment variable LOWD_BATCH_SHAPE=waves,prefetch,per_cu forces one
 * shape for every launch instead.  Arguments as for
 * lowd_batch_solve; the device arrays are copied, not kept.
 *   out  [host] out: the prepared batch; free with lowd_batch_free
 * Synchronises `stream`.
 */
lowd_status lowd_batch_prepare(int32_t G, const int64_t *node_ptr, const int64_t *edge_ptr,
                               const int32_t *src, const int32_t *dst, int32_t state,
                               int32_t star_max, int32_t tune, lowd_batch **out, void *stream);

/* lowd_batch_reset -- back to Algorithm 1's initial state, every graph
 * iterating again.  Synchronises `stream`. */
lowd_status lowd_batch_reset(lowd_batch *b, void *stream);

/*
 * lowd_batch_iterate -- `sweeps` more sweeps of every graph, continuing from
 * the current state, in one persistent launch (a HIP graph captured once
 * per distinct sweep count).  Asynchronous.
 */
lowd_status lowd_batch_iterate(lowd_batch *b, int32_t sweeps, void *stream);

/*
 * lowd_batch_extract -- every graph's densest set from its current loads
 * (Algorithm 1's extraction), and its largest load D_g, the dual bound of
 * Section III-B (rho_g <= rho*_g <= D_g).  The loads are FP64: for
 * LOWD_STATE_F32K, those of the graphs still iterating are recomputed from
 * the stored fractions, so that D_g is the bound of the fractions as stored
 * and not of the compensated loads the sweeps carry, and the carried loads
 * restart from them (a retired graph's fractions no longer change, and its
 * loads stay those of its last extraction).  Only the graphs still
 * iterating are extracted again; every array is written for all graphs, a
 * retired graph's entries being those of its last extraction.
 *   in_set  [device] uint8[total nodes] out
 *   num     [device] int64[G] out
 *   den     [device] int64[G] out
 *   D       [device] double[G] out, or NULL
 *   load    [device] double[total nodes] out (the FP64 loads above), or NULL
 * Asynchronous.
 */
lowd_status lowd_batch_extract(lowd_batch *b, uint8_t *in_set, int64_t *num, int64_t *den,
                               double *D, double *load, void *stream);

/*
 * lowd_batch_retire -- stops iterating the graphs that have converged: after
 * lowd_batch_extract, every graph whose relative gap (D_g - rho_g) / rho_g
 * (rho_g = num_g / den_g; a graph without edges counts as converged) is at
 * most tol leaves the set that later lowd_batch_iterate calls sweep; the
 * others keep their order (largest first).  lowd_batch_reset restores all.
 * A retired graph keeps its state, so its densest set and loads stay
 * available; its certified gap is at most tol.
 *   num, den, D   [device] the arrays the last lowd_batch_extract filled
 *   active        [host] out: graphs still iterating; may be NULL
 *   active_edges  [host] out: their edges; may be NULL
 * Synchronises `stream`.
 */
lowd_status lowd_batch_retire(lowd_batch *b, const int64_t *num, const int64_t *den,
                              const double *D, double tol, int32_t *active, int64_t *active_edges,
                              void *stream);

/*
 * lowd_batch_solve_prepared -- lowd_batch_solve on a prepared batch, from
 * its current state (lowd_batch_reset first for a fresh solve); the same
 * arguments from tol on.  Sweeps are counted from this call.
 */
lowd_status lowd_batch_solve_prepared(lowd_batch *b, double tol, int32_t max_sweeps,
                                      int32_t check_every, uint8_t *in_set, int64_t *num,
                                      int64_t *den, double *D, int32_t *sweeps_used,
                                      int32_t *set_sweeps, void *stream);

/*
 * lowd_batch_info --
 *   info [host] int64[9] out: G, total nodes, total edges, total phases,
 *        most phases of one graph, waves per workgroup, prefetching tile
 *        buffers (0/1), workgroups of the launch, LDS bytes per workgroup.
 */
lowd_status lowd_batch_info(const lowd_batch *b, int64_t *info);

/* Releases the prepared batch (waits for pending work).  NULL is accepted. */
void lowd_batch_free(lowd_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* LOWD_H */
