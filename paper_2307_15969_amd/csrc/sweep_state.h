// sweep_state.h -- the two solver states and the locally optimal step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "lowd_internal.h"

namespace lowd {

// Algorithm 1's step on edge e = (u, v) with u = src[e]: x = f_e(u) and
// f_e(v) = w - x.
//   if l_u > l_v: d = min((l_u - l_v)/2, f_e(u)); l_u -= d; f_e(u) -= d; l_v += d
//   else:         d = min((l_v - l_u)/2, f_e(v)); l_u += d; f_e(u) += d; l_v -= d
// When the else-branch moves the whole share (d == f_e(v)) the fraction is
// set to w exactly, so f_e(v) never becomes negative through rounding.  On
// l_u == l_v the else-branch runs with d = 0.  The library is compiled with
// -ffp-contract=off: every operation rounds on its own, as written.
//
// The kernels evaluate it without branches: both candidate moves are formed
// and selected, which performs the same FP64 operations on the same operands
// as the two-branch form (l_v - l_u equals -(l_u - l_v) exactly, so
// |l_u - l_v| * 0.5 is the else-branch's half), hence the same bits.  A
// chain of steps on one star then has no divergence between lanes.
struct StateF64 {
    using X = double;
    using L = double;
    using R = double;   // a load in registers
    static constexpr bool kRecompute = false;
    __host__ __device__ static inline X half_weight(float w) { return (double)w / 2.0; }
    __device__ static inline L infinite() { return __builtin_inf(); }
    __device__ static inline L from_f64(double v) { return v; }
    __device__ static inline double to_f64(L v) { return v; }
    __device__ static inline void step(L &lu, L &lv, X &x, float wf) {
        const double w = (double)wf;
        const double a = x;
        const double b = w - a;
        const double diff = lu - lv;
        const bool down = diff > 0.0;                 // l_u > l_v: move from u to v
        const double half = __builtin_fabs(diff) * 0.5;
        const double cap = down ? a : b;
        const double d = half < cap ? half : cap;
        const double lu_dn = lu - d, lu_up = lu + d;
        const double lv_dn = lv - d, lv_up = lv + d;
        const double x_dn = a - d, x_up = a + d;
        lu = down ? lu_dn : lu_up;
        lv = down ? lv_up : lv_dn;
        x = down ? x_dn : ((d == b) ? w : x_up);
    }
    // The same step written for a star, as the sweep kernels run it: lc is
    // the center's load, ll the leaf's; flip = 0x80000000 when the center is
    // v = dst (else 0).  u's excess over v is s = diff_c (center is u) or
    // -diff_c (center is v; exact negation by the sign bit), so the move goes
    // from u to v exactly when s > 0, its size is d = min(|s| * 0.5, cap),
    // and the center loses d exactly when that direction and the center's
    // role agree.  Both directions' moves are formed (d_dn = min(half, a),
    // d_up = min(half, b)) and applied, and the direction selects among the
    // results: the comparison then runs beside the arithmetic instead of
    // ahead of it, which shortens the dependent path from one step's center
    // load to the next's.  Only exact rewrites of step() are used: x - y ==
    // x + (-y); min picks one of its operands (none is NaN or -0 here);
    // negation flips the sign bit.  So the bits agree with step().
    __device__ static inline void step_center(L &lc, L &ll, uint32_t flip, X &x, float wf) {
        const double w = (double)wf;
        const double a = x;
        const double b = w - a;
        const double diff = lc - ll;
        const double half = __builtin_fabs(diff) * 0.5;
        const bool down = flip_sign(diff, flip) > 0.0;
        const double d_dn = min_f64(half, a);
        const double d_up = min_f64(half, b);
        // the center's change: down, it loses d_dn unless it is v; else it
        // gains d_up unless it is v
        const double c_dn = flip_sign(d_dn, 0x80000000u ^ flip);
        const double c_up = flip_sign(d_up, flip);
        const double lc_dn = lc + c_dn, lc_up = lc + c_up;
        const double ll_dn = ll - c_dn, ll_up = ll - c_up;
        lc = down ? lc_dn : lc_up;
        ll = down ? ll_dn : ll_up;
        x = down ? a - d_dn : ((d_up == b) ? w : a + d_up);
    }
    __device__ static inline double flip_sign(double v, uint32_t bit) {
        uint64_t u = __builtin_bit_cast(uint64_t, v) ^ ((uint64_t)bit << 32);
        return __builtin_bit_cast(double, u);
    }
    __device__ static inline double min_f64(double p, double q) {
        double r;
        asm("v_min_f64 %0, %1, %2" : "=v"(r) : "v"(p), "v"(q));
        return r;
    }
};

// FP32 fractions; loads stored as compensated FP32 pairs (s, c) with value
// s + c (s = the load rounded to FP32, c = the rest rounded to FP32: about
// 48 significant bits) wherever they rest in HBM: the station array and the
// batch's loads between launches (the LDS tiers keep them in FP64).
// A star's chain runs in FP64 registers: its loads are widened once when
// the tile reads them and rounded back to pairs once when it writes them,
// and each step is StateF64's step on the widened loads, with the fraction
// widened from FP32 and its new value rounded back to FP32.  So the
// dependent path of a step is FP64's, while the stored fractions take 4
// bytes.  The loads move by the step's exact d, the fractions by d rounded
// to FP32, so over many sweeps the carried loads can drift from the loads
// of the stored fractions (which alone form a feasible dual point); the
// checks recompute the latter in FP64 (kRecompute).
struct LoadK32 {
    float s, c;
};

struct StateF32K {
    using X = float;
    using L = LoadK32;
    using R = double;
    static constexpr bool kRecompute = true;
    __host__ __device__ static inline X half_weight(float w) { return w * 0.5f; }
    __device__ static inline L infinite() { return L{__builtin_inff(), 0.0f}; }
    // the pair of v: s = v rounded to FP32, c = (v - s) rounded to FP32
    // (v - s is exact in FP64); an infinite v (the padding leaf, whose entry
    // the node form writes back) keeps c = 0
    __device__ static inline L from_f64(double v) {
        L r;
        r.s = (float)v;
        const float c = (float)(v - (double)r.s);
        r.c = __builtin_isinf(r.s) ? 0.0f : c;
        return r;
    }
    __device__ static inline double to_f64(L v) { return (double)v.s + (double)v.c; }
    __device__ static inline void step_center(R &lc, R &ll, uint32_t flip, X &x, float w) {
        double xd = (double)x;
        StateF64::step_center(lc, ll, flip, xd, w);
        x = (float)xd;
    }
};

// Arguments of the batched solve in one launch (k_batch_solve): the graphs,
// their layouts and state, the batch's incidence for the checks, per-node
// scratch of the checks (each graph owns its nodes' slice), the tolerance
// and the per-graph results.
struct BatchSolveArgs {
    const int32_t *active;        // [1] graphs listed in order
    const int32_t *order;         // [G] graph ids, largest first
    unsigned *queue;              // [2] next list index; graphs that reached max_sweeps
    const int64_t *node_ptr;      // [G+1]
    const int64_t *desc_ptr;      // [G+1]
    const PhaseDesc *descs;
    const int32_t *tile_center;
    const uint32_t *slot_leaf;
    void *slot_x;
    void *Lstate;                 // [N] carried loads, read at the start, written at the end
    const int64_t *row_ptr;       // [N+1] incidence rows (ascending edge index)
    const int32_t *adj;           // [2M] the other end of each entry (batch node id)
    const uint32_t *inc_slot;     // [2M] slot << 1 | side of each entry (FP32K)
    uint64_t *k0, *k1;            // [N] sort keys
    uint32_t *i0, *i1;            // [N] sort ids
    int32_t *pos, *hist;          // [N] positions, edge counts by position
    double tol;
    int32_t max_sweeps, check_every;
    uint8_t *in_set;              // [N] out
    int64_t *num, *den;           // [G] out
    double *D;                    // [G] out
    int32_t *sweeps_used;         // [G] out
    int32_t *set_sweeps;          // [G] out: the sweep count of the set's extraction
};

// (D - rho) / rho for rho = num / den (a graph without edges: 0)
__host__ __device__ inline double batch_rel_gap(double D, int64_t num, int64_t den) {
    const double rho = den > 0 ? (double)num / (double)den : 0.0;
    return rho > 0.0 ? (D - rho) / rho : (D > 0.0 ? 1.0e300 : 0.0);
}

// A load in FP64 from its stored form, and back: the LDS tiers hold FP64
// loads for either state (LDS is private to the run: the pair form is kept
// only where loads rest in HBM between phases and launches).
__device__ inline double widen(double v) { return v; }
__device__ inline double widen(LoadK32 v) { return StateF32K::to_f64(v); }
template <class T>
__device__ inline T narrow(double v);
template <>
__device__ inline double narrow<double>(double v) { return v; }
template <>
__device__ inline LoadK32 narrow<LoadK32>(double v) { return StateF32K::from_f64(v); }

// Host-callable launchers for one (state, weighted) combination.
struct SweepLaunch {
    void (*init_slots)(int64_t nslots, const int64_t *slot_edge, const float *w, void *slot_x,
                       float *slot_w, hipStream_t s);
    // big[nbig]: the nodes of degree >= kBigRow (a wave or workgroup each)
    void (*init_loads)(int32_t n, const int64_t *row_ptr, const uint32_t *inc, const float *w,
                       const uint32_t *home, const int32_t *big, int32_t nbig, int64_t entries,
                       int64_t center_base, void *E, hipStream_t s);
    // slot_src / center_src: NULL for a pushed phase; for a pulled one the
    // entries its slots and lanes read (Schedule::slot_src, center_src)
    void (*phase)(const PhaseDescWide &d, int64_t center_base, const uint32_t *center_next,
                  const uint32_t *slot_next, void *slot_x, const float *slot_w, void *E,
                  const uint32_t *slot_src, const uint32_t *center_src, hipStream_t s);
    // the node form (loads in a node-indexed array; whole-GPU phases only)
    void (*phase_node)(const PhaseDescWide &d, const int32_t *tile_center,
                       const uint32_t *slot_leaf, void *slot_x, const float *slot_w, void *E,
                       hipStream_t s);
    void (*fill_nodes)(int32_t n, void *E, hipStream_t s);
    void (*tail)(int32_t nph, const PhaseDesc *descs, const int32_t *tile_center,
                 const uint32_t *slot_leaf, void *slot_x, const float *slot_w, int64_t tail_base,
                 const uint32_t *tail_next, int32_t ntail, void *E, hipStream_t s);
    void (*mid)(int32_t nph, const PhaseDesc *descs, int64_t center_base,
                const uint32_t *center_next, const uint32_t *slot_next, void *slot_x,
                const float *slot_w, void *E, hipStream_t s);
    void (*set_tail_lds)(size_t bytes);
    void (*set_mid_lds)(size_t bytes);
    void (*loads_f64)(int32_t n, const int64_t *row_ptr, const uint32_t *inc,
                      const int64_t *edge_slot, const void *slot_x, const float *w,
                      const uint32_t *home, const int32_t *big, int32_t nbig, const void *E,
                      double *L64, hipStream_t s);
    void (*write_loads)(int32_t n, const uint32_t *home, const double *L64, void *E,
                        hipStream_t s);
    void (*read_x)(int64_t m, const int64_t *edge_slot, const void *slot_x, double *x,
                   hipStream_t s);
    void (*read_loads)(int32_t n, const uint32_t *home, const void *E, double *out,
                       hipStream_t s);
    // the batched form; shape = 2 * waves per workgroup (4 or 8) + prefetch (0/1)
    void (*batch)(int32_t shape, const int32_t *active, const int32_t *order, unsigned *queue,
                  const int64_t *node_ptr, const int64_t *desc_ptr, const PhaseDesc *descs,
                  const int32_t *tile_center, const uint32_t *slot_leaf, void *slot_x,
                  int32_t sweeps, void *Lstate, size_t lds, int32_t blocks, hipStream_t s);
    void (*set_batch_lds)(int32_t shape, size_t bytes);
    // the batched solve in one launch (same shapes as batch)
    void (*batch_solve)(int32_t shape, const BatchSolveArgs &a, size_t lds, int32_t blocks,
                        hipStream_t s);
    void (*set_batch_solve_lds)(int32_t shape, size_t bytes);
    void (*batch_init_loads)(int64_t N, const int32_t *deg, void *Lstate, hipStream_t s);
    void (*batch_loads_f64)(int64_t N, const void *Lstate, double *L64, hipStream_t s);
    void (*batch_recompute)(int32_t G, int64_t N, const int32_t *active, const int32_t *order,
                            const int32_t *node_graph, uint8_t *flag, const int64_t *row_ptr,
                            const uint32_t *inc, const int64_t *edge_slot, const void *slot_x,
                            double *L64, void *Lstate, hipStream_t s);
    size_t x_bytes;
    size_t l_bytes;
};

void get_sweep_launchers(int32_t state, bool weighted, SweepLaunch &fn);
void launch_stats(int64_t n, const double *L64, double *partial, int32_t nb, double *out,
                  hipStream_t s);
// batches: node degrees (once per batch)
void launch_batch_degrees(int64_t N, int64_t M, const int32_t *gsrc, const int32_t *gdst,
                          int32_t *deg, hipStream_t s);
// batches: keep the graphs (of `all`, in order) whose gap exceeds tol, or all
void launch_retire(int32_t G, const int32_t *all, const int64_t *edge_ptr, const int64_t *num,
                   const int64_t *den, const double *D, double tol, int32_t *order,
                   int32_t *active, int64_t *active_edges, hipStream_t s);
// inc_slot[j] = edge_slot[inc[j] >> 1] << 1 | (inc[j] & 1)
void launch_inc_slots(int64_t entries, const uint32_t *inc, const int64_t *edge_slot,
                      uint32_t *inc_slot, hipStream_t s);
void launch_activate_all(int32_t G, const int32_t *all, const int64_t *edge_ptr, int32_t *order,
                         int32_t *active, int64_t *active_edges, hipStream_t s);

}  // namespace lowd
