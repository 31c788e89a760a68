/*
 * oracle.c -- plain sequential FP64 reference of the LOWD densest-subgraph
 * method (Zhu, Liu, Feng, Cheng, "Fast Searching The Densest Subgraph And
 * Decomposition With Local Optimality", arXiv 2307.15969).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no source,
 * header, table or helper with the GPU library: it is written from the paper,
 * slowly and literally, so that a reader can check it against the paper.
 *
 * Build: gcc -O2 -ffp-contract=off -fPIC -shared (no fused multiply-add may
 * be formed: the per-edge step must round exactly as written).
 *
 * Graph convention (Section II, Problem 1): nodes 0..n-1, m undirected edges
 * (src[e], dst[e]) with src != dst and no repeated pair; weight w[e] > 0, or
 * w == NULL for an unweighted graph (every w_e = 1).  The weights are given
 * as float32 (the GPU path reads the same float32 values) and widened to
 * FP64 here.
 *
 * Readings of the paper where it is silent (each also listed in the design
 * notes):
 *  - one edge fraction is stored per edge: x[e] = f_e(src[e]); the other
 *    endpoint's share is w_e - x[e], so f_e(u) + f_e(v) = w_e holds exactly
 *    (tighter dual LP, Section III-B);
 *  - the per-edge step is the d-form of Algorithm 1 with (a-b)*0.5; on a tie
 *    l_u == l_v the else-branch runs with d = 0; when the else-branch moves
 *    the whole share (d == w_e - x[e]) x[e] is set to w_e exactly;
 *  - the edge order of a sweep is an input (Algorithm 1 iterates "for e in E"
 *    without an order; Fig. 1 notes the order does not change the limit);
 *  - initial loads sum each node's incident shares in ascending edge index;
 *  - the load sort is stable ascending on (load, node id); the empty set is
 *    never a candidate; the largest prefix of maximal density is kept
 *    (S* starts as V and is replaced only on a strict increase);
 *  - pruning removes, each round, every node whose degree is below the
 *    current density, then recomputes the density (Algorithm 2);
 *  - densities W(S)/|S| (Problem 1) are compared exactly, also for
 *    weighted graphs: the float32 weights are exact binary fractions, so
 *    their sums are taken as exact integers in a common unit.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 oracle_u128;

#define ORACLE_OK 0
#define ORACLE_E_ARG (-1)
#define ORACLE_E_NOMEM (-2)

static double weight_of(const float *w, int64_t e) { return w ? (double)w[e] : 1.0; }

/* ------------------------------------------------------------------------ *
 * Algorithm 2 (Pruning), unweighted graphs.
 *   H <- G; delta <- rho(H);
 *   while some nodes of H have degree in H below delta:
 *       remove all of them and their edges; delta <- rho(H)
 * Degrees are recomputed from scratch every round (plain, O(M) per round).
 * A node u is removed when deg_H(u) < |E(H)| / |V(H)|, decided exactly in
 * integers as deg_H(u) * |V(H)| < |E(H)|.  Isolated nodes count in |V(H)|.
 * ------------------------------------------------------------------------ */
int oracle_prune(int64_t n, int64_t m, const int32_t *src, const int32_t *dst,
                 uint8_t *node_keep, int32_t *rounds_out, int64_t *n_h_out, int64_t *m_h_out)
{
    if (n < 0 || m < 0 || !node_keep) return ORACLE_E_ARG;
    int64_t *deg = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    if (!deg) return ORACLE_E_NOMEM;
    for (int64_t u = 0; u < n; ++u) node_keep[u] = 1;
    int32_t rounds = 0;
    int64_t N = n, M = m;
    for (;;) {
        /* |V(H)| and |E(H)| and the degrees in H, from scratch */
        N = 0;
        for (int64_t u = 0; u < n; ++u) { deg[u] = 0; N += node_keep[u]; }
        M = 0;
        for (int64_t e = 0; e < m; ++e) {
            if (node_keep[src[e]] && node_keep[dst[e]]) {
                ++M;
                ++deg[src[e]];
                ++deg[dst[e]];
            }
        }
        /* the set H' of nodes below the density of H */
        int64_t removed = 0;
        for (int64_t u = 0; u < n; ++u)
            if (node_keep[u] && deg[u] * N < M) ++removed;
        if (removed == 0) break;
        for (int64_t u = 0; u < n; ++u)
            if (node_keep[u] && deg[u] * N < M) node_keep[u] = 0;
        ++rounds;
    }
    if (rounds_out) *rounds_out = rounds;
    if (n_h_out) *n_h_out = N;
    if (m_h_out) *m_h_out = M;
    free(deg);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ *
 * Edge schedule (not part of the paper: it fixes the edge order that
 * Algorithm 1 leaves open).  Edges are split into phases; inside a phase the
 * edges form vertex-disjoint stars, so the stars can be processed at the same
 * time while the result equals processing the phase's edges one by one.
 *
 * Definition:
 *   deg(u)  = number of edges at u;
 *   center  of edge e = the endpoint of larger degree, ties to the smaller id;
 *   leaf    = the other endpoint;
 *   key(e)  = the e-th output (counting from 0) of SplitMix64 seeded with 0
 *             (Steele, Lea, Flood 2014): the generator adds 0x9E3779B97F4A7C15
 *             to its state, then mixes: z ^= z >> 30, z *= 0xBF58476D1CE4E5B9,
 *             z ^= z >> 27, z *= 0x94D049BB133111EB, z ^= z >> 31;
 *   edges are visited by ascending key, ties by ascending index; edge e goes
 *   to the smallest phase p in which its center is not a leaf and is the
 *   center of fewer than smax leaves, and its leaf does not appear at all.
 * Sequential order: ascending (phase, edge index).
 *
 * Plain implementation: one byte per (node, phase):
 *   0 = absent, 255 = leaf, k in 1..254 = center of k leaves.
 * phase_out[e], center_out[e] (the center node of e) and order_out[m] are
 * written; *nphases_out = number of phases.
 * ------------------------------------------------------------------------ */
/* SplitMix64: the output after the state has advanced `steps` times from 0 */
static uint64_t splitmix64_output(uint64_t steps)
{
    uint64_t state = 0;
    state += steps * 0x9E3779B97F4A7C15ull;   /* `steps` additions of the increment */
    uint64_t z = state;
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}

static const uint64_t *g_sort_key;
static int cmp_key_then_index(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    if (g_sort_key[a] != g_sort_key[b]) return g_sort_key[a] < g_sort_key[b] ? -1 : 1;
    return (a > b) - (a < b);
}

int oracle_schedule(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, int32_t smax,
                    int32_t *phase_out, int32_t *center_out, int32_t *order_out, int32_t *nphases_out)
{
    if (n < 0 || m < 0 || smax < 1 || smax > 254) return ORACLE_E_ARG;
    int64_t *deg = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    uint8_t **role = (uint8_t **)calloc((size_t)(n > 0 ? n : 1), sizeof(uint8_t *));
    int32_t *len = (int32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
    if (!deg || !role || !len) { free(deg); free(role); free(len); return ORACLE_E_NOMEM; }
    for (int64_t e = 0; e < m; ++e) { ++deg[src[e]]; ++deg[dst[e]]; }
    /* orientation and visiting order */
    int32_t *ctr = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    int32_t *lf = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    uint64_t *key = (uint64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(uint64_t));
    int64_t *visit = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    if (!ctr || !lf || !key || !visit) {
        free(ctr); free(lf); free(key); free(visit); free(deg); free(role); free(len);
        return ORACLE_E_NOMEM;
    }
    for (int64_t e = 0; e < m; ++e) {
        int32_t a = src[e], b = dst[e];
        if (deg[a] > deg[b] || (deg[a] == deg[b] && a < b)) { ctr[e] = a; lf[e] = b; }
        else { ctr[e] = b; lf[e] = a; }
        key[e] = splitmix64_output((uint64_t)e + 1);   /* the e-th output, from 0 */
        visit[e] = e;
    }
    g_sort_key = key;
    qsort(visit, (size_t)m, sizeof(int64_t), cmp_key_then_index);
    int32_t P = 0;
    int rc = ORACLE_OK;
    for (int64_t i = 0; i < m && rc == ORACLE_OK; ++i) {
        const int64_t e = visit[i];
        const int32_t c = ctr[e], l = lf[e];
        int32_t p = 0;
        for (;; ++p) {
            uint8_t rc_ = p < len[c] ? role[c][p] : 0;
            uint8_t rl_ = p < len[l] ? role[l][p] : 0;
            int center_ok = (rc_ == 0) || (rc_ != 255 && rc_ < smax);
            int leaf_ok = (rl_ == 0);
            if (center_ok && leaf_ok) break;
        }
        /* grow both role arrays to cover phase p */
        int32_t who[2] = {c, l};
        for (int k = 0; k < 2; ++k) {
            int32_t u = who[k];
            if (p >= len[u]) {
                int32_t nl = p + 1 + (p >> 1) + 8;
                uint8_t *r = (uint8_t *)realloc(role[u], (size_t)nl);
                if (!r) { rc = ORACLE_E_NOMEM; break; }
                memset(r + len[u], 0, (size_t)(nl - len[u]));
                role[u] = r;
                len[u] = nl;
            }
        }
        if (rc != ORACLE_OK) break;
        role[c][p] = (uint8_t)(role[c][p] + 1);
        role[l][p] = 255;
        phase_out[e] = p;
        if (center_out) center_out[e] = c;
        if (p + 1 > P) P = p + 1;
    }
    for (int64_t u = 0; u < n; ++u) free(role[u]);
    free(role); free(len); free(deg);
    free(ctr); free(lf); free(key); free(visit);
    if (rc != ORACLE_OK) return rc;
    /* order: ascending (phase, edge index), by counting */
    if (order_out) {
        int64_t *start = (int64_t *)calloc((size_t)P + 1, sizeof(int64_t));
        if (!start) return ORACLE_E_NOMEM;
        for (int64_t e = 0; e < m; ++e) ++start[phase_out[e] + 1];
        for (int32_t p = 0; p < P; ++p) start[p + 1] += start[p];
        for (int64_t e = 0; e < m; ++e) order_out[start[phase_out[e]]++] = (int32_t)e;
        free(start);
    }
    if (nphases_out) *nphases_out = P;
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ *
 * Algorithm 1, initialisation: f_e(u) = f_e(v) = w_e / 2 and
 * l_u = sum of f_e(u) over the edges at u (ascending edge index, from 0).
 * ------------------------------------------------------------------------ */
int oracle_init(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const float *w,
                double *x, double *L)
{
    if (n < 0 || m < 0) return ORACLE_E_ARG;
    for (int64_t u = 0; u < n; ++u) L[u] = 0.0;
    for (int64_t e = 0; e < m; ++e) {
        double we = weight_of(w, e);
        x[e] = we / 2.0;
        L[src[e]] = L[src[e]] + x[e];
        L[dst[e]] = L[dst[e]] + (we - x[e]);
    }
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ *
 * Algorithm 1, the locally optimal step on one edge e = (u, v), u = src[e]:
 *   if l_u > l_v:  d = min((l_u - l_v)/2, f_e(u)); move d from u to v
 *   else:          d = min((l_v - l_u)/2, f_e(v)); move d from v to u
 * with f_e(u) = x[e], f_e(v) = w_e - x[e].
 * ------------------------------------------------------------------------ */
static void lowd_step(int32_t u, int32_t v, double we, double *xe, double *L)
{
    double a = *xe;          /* f_e(u) */
    double b = we - a;       /* f_e(v) */
    if (L[u] > L[v]) {
        double half = (L[u] - L[v]) * 0.5;
        double d = half < a ? half : a;
        L[u] = L[u] - d;
        *xe = a - d;
        L[v] = L[v] + d;
    } else {
        double half = (L[v] - L[u]) * 0.5;
        double d = half < b ? half : b;
        L[u] = L[u] + d;
        *xe = (d == b) ? we : a + d;
        L[v] = L[v] - d;
    }
}

/* T sweeps; each sweep applies the step to order[0], order[1], ...,
 * order[k-1] in that sequence (k may be smaller than m for a partial pass). */
int oracle_sweep(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const float *w,
                 const int32_t *order, int64_t k, int32_t T, double *x, double *L)
{
    (void)n;
    if (k < 0 || k > m || T < 0) return ORACLE_E_ARG;
    for (int32_t t = 0; t < T; ++t)
        for (int64_t i = 0; i < k; ++i) {
            int32_t e = order[i];
            lowd_step(src[e], dst[e], weight_of(w, e), &x[e], L);
        }
    return ORACLE_OK;
}

/* D = max load, sum of loads, sum of squared loads (QP objective). */
int oracle_stats(int64_t n, const double *L, double *D, double *sumL, double *sumL2)
{
    double mx = n > 0 ? L[0] : 0.0, s = 0.0, s2 = 0.0;
    for (int64_t u = 0; u < n; ++u) {
        if (L[u] > mx) mx = L[u];
        s = s + L[u];
        s2 = s2 + L[u] * L[u];
    }
    if (D) *D = mx;
    if (sumL) *sumL = s;
    if (sumL2) *sumL2 = s2;
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ *
 * Exact weights.  A positive finite float32 w is M * 2^E for an odd integer
 * M < 2^24 (frexpf gives w = f * 2^e with f in [0.5, 1); M = f * 2^24 is an
 * integer, then trailing zero bits move into E).  With q = the smallest E
 * over the edges, w / 2^q = M * 2^(E - q) is an integer.  Sums of such
 * integers are exact; W / 2^q values are returned as FP64 once, by
 * ldexp((double) W, q).  Fails (ORACLE_E_ARG) if an integer would not fit
 * 64 bits.  *wi is malloc'ed (m entries).
 * ------------------------------------------------------------------------ */
static int exact_weights(int64_t m, const float *w, uint64_t **wi_out, int *q_out)
{
    int64_t *E = (int64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int64_t));
    uint64_t *M = (uint64_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(uint64_t));
    if (!E || !M) { free(E); free(M); return ORACLE_E_NOMEM; }
    int q = 0;
    for (int64_t e = 0; e < m; ++e) {
        int ex = 0;
        float f = frexpf(w[e], &ex);
        uint64_t mm = (uint64_t)ldexpf(f, 24);
        int64_t ee = (int64_t)ex - 24;
        while (mm != 0 && (mm & 1) == 0) { mm >>= 1; ++ee; }
        M[e] = mm;
        E[e] = ee;
        if (e == 0 || ee < q) q = (int)ee;
    }
    for (int64_t e = 0; e < m; ++e) {
        int64_t sh = E[e] - q;
        if (sh > 40) { free(E); free(M); return ORACLE_E_ARG; }
        M[e] <<= sh;
    }
    free(E);
    *wi_out = M;
    *q_out = q;
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ *
 * Algorithm 1, extraction: V_s = nodes sorted by load, non-decreasing
 * (stable: equal loads by ascending id); S_i = V minus its first i nodes;
 * S* = the S_i (0 <= i < n) of largest density, first (largest) on ties.
 *
 * W(S_i) = total weight of edges with both ends in S_i: an edge is inside
 * S_i exactly when min(pos_u, pos_v) >= i, so W is the suffix sum of the
 * weights binned at min(pos_u, pos_v).  W is an exact integer (unit
 * weights: an edge count; weighted: in units of 2^q, see exact_weights),
 * and densities are compared exactly by cross-multiplication.
 * Outputs: in_set[n] (1 = in S*), *best_i, *num_unit (W for unit weights),
 * *num_w (W as FP64, rounded once), *den (|S*|).
 * ------------------------------------------------------------------------ */
static const double *g_sort_L;
static int cmp_load_then_id(const void *pa, const void *pb)
{
    int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    if (g_sort_L[a] < g_sort_L[b]) return -1;
    if (g_sort_L[a] > g_sort_L[b]) return 1;
    return (a > b) - (a < b);
}

int oracle_extract(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const float *w,
                   const double *L, uint8_t *in_set, int64_t *best_i_out, int64_t *num_unit,
                   double *num_w, int64_t *den)
{
    if (n <= 0) return ORACLE_E_ARG;
    uint64_t *wi = NULL;
    int q = 0;
    if (w) {
        int rc = exact_weights(m, w, &wi, &q);
        if (rc != ORACLE_OK) return rc;
    }
    int32_t *asc = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int64_t *pos = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    oracle_u128 *W = (oracle_u128 *)calloc((size_t)n + 1, sizeof(oracle_u128));
    if (!asc || !pos || !W) { free(asc); free(pos); free(W); free(wi); return ORACLE_E_NOMEM; }
    for (int64_t u = 0; u < n; ++u) asc[u] = (int32_t)u;
    g_sort_L = L;
    qsort(asc, (size_t)n, sizeof(int32_t), cmp_load_then_id);
    for (int64_t i = 0; i < n; ++i) pos[asc[i]] = i;
    for (int64_t e = 0; e < m; ++e) {
        int64_t t = pos[src[e]] < pos[dst[e]] ? pos[src[e]] : pos[dst[e]];
        W[t] += w ? (oracle_u128)wi[e] : 1;
    }
    for (int64_t i = n - 1; i >= 0; --i) W[i] += W[i + 1];
    int64_t best = 0;
    for (int64_t i = 1; i < n; ++i)
        if (W[best] * (oracle_u128)(n - i) < W[i] * (oracle_u128)(n - best)) best = i;
    for (int64_t u = 0; u < n; ++u) in_set[u] = pos[u] >= best ? 1 : 0;
    if (best_i_out) *best_i_out = best;
    if (num_unit) *num_unit = w ? 0 : (int64_t)W[best];
    if (num_w) *num_w = ldexp((double)W[best], q);
    if (den) *den = n - best;
    free(asc); free(pos); free(W); free(wi);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ *
 * Locally-dense decomposition read from a load vector (Problem 2, Property
 * 2).  The nodes are ranked by descending load: the reverse of the
 * extraction's stable ascending order on (load, id).  Only prefixes of that
 * ranking are candidate sets.  Let f(k) be the weight of the edges with
 * both endpoints among the top k nodes (f(0) = 0).  Then, as in the
 * definition of B_i, starting from k_0 = 0:
 *     k_j = the largest k > k_{j-1} maximising
 *           (f(k) - f(k_{j-1})) / (k - k_{j-1}),
 * until k_j = n.  Level j-1 holds the nodes of rank k_{j-1} .. k_j - 1, and
 * lambda_j is that maximal ratio.  At the limit of the iteration the
 * ranking is consistent with the decomposition and this is the exact LDD.
 * The ratios are compared exactly by cross-multiplication of integers (edge
 * counts, or weights in units of 2^q, see exact_weights); f_end holds f
 * rounded once to FP64.
 *   level  [n]  out: level of each node (0 = densest)
 *   k_end  [n]  out: k_1 .. k_L (L levels)
 *   f_end  [n]  out: f(k_1) .. f(k_L)
 * ------------------------------------------------------------------------ */
int oracle_ldd(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, const float *w,
               const double *L, int32_t *level, int64_t *k_end, double *f_end, int64_t *nlevels)
{
    if (n <= 0 || !level || !k_end || !f_end || !nlevels) return ORACLE_E_ARG;
    uint64_t *wi = NULL;
    int q = 0;
    if (w) {
        int rc = exact_weights(m, w, &wi, &q);
        if (rc != ORACLE_OK) return rc;
    }
    int32_t *asc = (int32_t *)malloc((size_t)n * sizeof(int32_t));
    int64_t *rank = (int64_t *)malloc((size_t)n * sizeof(int64_t));
    oracle_u128 *f = (oracle_u128 *)calloc((size_t)n + 1, sizeof(oracle_u128));
    if (!asc || !rank || !f) { free(asc); free(rank); free(f); free(wi); return ORACLE_E_NOMEM; }
    for (int64_t u = 0; u < n; ++u) asc[u] = (int32_t)u;
    g_sort_L = L;
    qsort(asc, (size_t)n, sizeof(int32_t), cmp_load_then_id);
    for (int64_t i = 0; i < n; ++i) rank[asc[i]] = n - 1 - i;
    /* an edge is inside the top k exactly when k > the larger rank of its ends */
    for (int64_t e = 0; e < m; ++e) {
        int64_t r = rank[src[e]] > rank[dst[e]] ? rank[src[e]] : rank[dst[e]];
        f[r + 1] += w ? (oracle_u128)wi[e] : 1;
    }
    for (int64_t k = 1; k <= n; ++k) f[k] += f[k - 1];
    int64_t L_count = 0, kp = 0;
    while (kp < n) {
        int64_t best = kp + 1;
        for (int64_t k = kp + 2; k <= n; ++k) {
            /* (f(k)-f(kp))/(k-kp) >= (f(best)-f(kp))/(best-kp), exactly */
            oracle_u128 a = (f[k] - f[kp]) * (oracle_u128)(best - kp);
            oracle_u128 b = (f[best] - f[kp]) * (oracle_u128)(k - kp);
            if (a >= b) best = k;
        }
        k_end[L_count] = best;
        f_end[L_count] = ldexp((double)f[best], q);
        for (int64_t i = 0; i < n; ++i)
            if (rank[i] >= kp && rank[i] < best) level[i] = (int32_t)L_count;
        ++L_count;
        kp = best;
    }
    *nlevels = L_count;
    free(asc); free(rank); free(f); free(wi);
    return ORACLE_OK;
}

/* ------------------------------------------------------------------------ *
 * Greedy peeling (Appendix, Algorithm 3) on an unweighted graph: starting
 * from S = V and S* = V, repeatedly remove a node of minimum degree in S
 * (ties: the smallest id) with its edges; after each removal, if
 * rho(S) > rho(S*) then S* = S.  Plain: every step scans all nodes.
 *   order  [n]  out: the removal order
 *   rem_m  [n]  out: |E(S)| after each removal
 *   *best_i     out: the number of removals before S* (0 = V)
 * ------------------------------------------------------------------------ */
int oracle_greedy(int64_t n, int64_t m, const int32_t *src, const int32_t *dst, int32_t *order,
                  int64_t *rem_m, int64_t *best_i)
{
    if (n <= 0 || !order || !rem_m || !best_i) return ORACLE_E_ARG;
    int64_t *deg = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    uint8_t *alive = (uint8_t *)malloc((size_t)n);
    int64_t *rp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *adj = (int32_t *)malloc((size_t)(m > 0 ? 2 * m : 1) * sizeof(int32_t));
    if (!deg || !alive || !rp || !adj) { free(deg); free(alive); free(rp); free(adj); return ORACLE_E_NOMEM; }
    for (int64_t e = 0; e < m; ++e) { ++rp[src[e] + 1]; ++rp[dst[e] + 1]; }
    for (int64_t u = 0; u < n; ++u) rp[u + 1] += rp[u];
    {
        int64_t *fill = (int64_t *)malloc((size_t)n * sizeof(int64_t));
        if (!fill) { free(deg); free(alive); free(rp); free(adj); return ORACLE_E_NOMEM; }
        for (int64_t u = 0; u < n; ++u) fill[u] = rp[u];
        for (int64_t e = 0; e < m; ++e) { adj[fill[src[e]]++] = dst[e]; adj[fill[dst[e]]++] = src[e]; }
        free(fill);
    }
    for (int64_t u = 0; u < n; ++u) { deg[u] = rp[u + 1] - rp[u]; alive[u] = 1; }
    int64_t M = m, N = n, bestM = m, bestN = n;
    *best_i = 0;
    for (int64_t step = 0; step < n; ++step) {
        int64_t u = -1;
        for (int64_t v = 0; v < n; ++v)
            if (alive[v] && (u < 0 || deg[v] < deg[u])) u = v;
        order[step] = (int32_t)u;
        alive[u] = 0;
        M -= deg[u];
        N -= 1;
        for (int64_t j = rp[u]; j < rp[u + 1]; ++j)
            if (alive[adj[j]]) --deg[adj[j]];
        rem_m[step] = M;
        /* M / N > bestM / bestN, exactly */
        if (N > 0 && (__int128)M * bestN > (__int128)bestM * N) {
            bestM = M;
            bestN = N;
            *best_i = step + 1;
        }
    }
    free(deg); free(alive); free(rp); free(adj);
    return ORACLE_OK;
}
