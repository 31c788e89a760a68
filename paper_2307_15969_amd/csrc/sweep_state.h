// sweep_state.h -- the two solver states and the locally optimal step.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lowd {

// Algorithm 1's step on edge e = (u, v) with u = src[e]: x = f_e(u) and
// f_e(v) = w - x.
//   if l_u > l_v: d = min((l_u - l_v)/2, f_e(u)); l_u -= d; f_e(u) -= d; l_v += d
//   else:         d = min((l_v - l_u)/2, f_e(v)); l_u += d; f_e(u) += d; l_v -= d
// When the else-branch moves the whole share (d == f_e(v)) the fraction is
// set to w exactly, so f_e(v) never becomes negative through rounding.  On
// l_u == l_v the else-branch runs with d = 0.  The library is compiled with
// -ffp-contract=off: every operation rounds on its own, as written.
struct StateF64 {
    using X = double;
    using L = double;
    static constexpr bool kRecompute = false;
    __host__ __device__ static inline X half_weight(float w) { return (double)w / 2.0; }
    __device__ static inline L from_f64(double v) { return v; }
    __device__ static inline double to_f64(L v) { return v; }
    __device__ static inline void step(L &lu, L &lv, X &x, float wf) {
        const double w = (double)wf;
        const double a = x;
        const double b = w - a;
        if (lu > lv) {
            const double half = (lu - lv) * 0.5;
            const double d = half < a ? half : a;
            lu = lu - d;
            x = a - d;
            lv = lv + d;
        } else {
            const double half = (lv - lu) * 0.5;
            const double d = half < b ? half : b;
            lu = lu + d;
            x = (d == b) ? w : a + d;
            lv = lv - d;
        }
    }
};

// FP32 fractions; FP32 loads carried as (s, c) with value s + c, where every
// addition to a load is exact-error compensated (two-sum: the rounding error
// of s + y is accumulated into c).  Differences of loads are taken as
// (s_u - s_v) + (c_u - c_v).
struct LoadK32 {
    float s, c;
};

struct StateF32K {
    using X = float;
    using L = LoadK32;
    static constexpr bool kRecompute = true;
    __host__ __device__ static inline X half_weight(float w) { return w * 0.5f; }
    __device__ static inline L from_f64(double v) {
        L r;
        r.s = (float)v;
        r.c = (float)(v - (double)r.s);
        return r;
    }
    __device__ static inline double to_f64(L v) { return (double)v.s + (double)v.c; }
    __device__ static inline void add(L &a, float y) {
        const float t = a.s + y;
        const float z = t - a.s;
        const float e = (a.s - (t - z)) + (y - z);
        a.s = t;
        a.c = a.c + e;
    }
    __device__ static inline void step(L &lu, L &lv, X &x, float w) {
        const float a = x;
        const float b = w - a;
        const float diff = (lu.s - lv.s) + (lu.c - lv.c);
        if (diff > 0.0f) {
            const float half = diff * 0.5f;
            const float d = half < a ? half : a;
            add(lu, -d);
            x = a - d;
            add(lv, d);
        } else {
            const float half = -diff * 0.5f;
            const float d = half < b ? half : b;
            add(lu, d);
            x = (d == b) ? w : a + d;
            add(lv, -d);
        }
    }
};

// Host-callable launchers for one (state, weighted) combination.
struct SweepLaunch {
    void (*init_slots)(int64_t nslots, const int64_t *slot_edge, const float *w, void *slot_x,
                       float *slot_w, hipStream_t s);
    void (*init_loads)(int32_t n, const int64_t *row_ptr, const uint32_t *inc, const float *w,
                       void *L, hipStream_t s);
    void (*phase)(int32_t t0, int32_t t1, const int32_t *tile_center, const int64_t *tile_base,
                  const int32_t *tile_depth, const uint32_t *slot_leaf, void *slot_x,
                  const float *slot_w, void *L, hipStream_t s);
    void (*tail)(int32_t nph, const int32_t *ph_tile_ptr, const int32_t *tile_center,
                 const int64_t *tile_base, const int32_t *tile_depth, const uint32_t *slot_leaf,
                 void *slot_x, const float *slot_w, const int32_t *tail_nodes, int32_t ntail,
                 void *L, hipStream_t s);
    void (*set_tail_lds)(size_t bytes);
    void (*loads_f64)(int32_t n, const int64_t *row_ptr, const uint32_t *inc,
                      const int64_t *edge_slot, const void *slot_x, const float *w, const void *L,
                      double *L64, hipStream_t s);
    void (*read_x)(int64_t m, const int64_t *edge_slot, const void *slot_x, double *x,
                   hipStream_t s);
    void (*read_loads)(int32_t n, const void *L, double *out, hipStream_t s);
    size_t x_bytes;
    size_t l_bytes;
};

void get_sweep_launchers(int32_t state, bool weighted, SweepLaunch &fn);
void launch_stats(int64_t n, const double *L64, double *partial, int32_t nb, double *out,
                  hipStream_t s);

}  // namespace lowd
