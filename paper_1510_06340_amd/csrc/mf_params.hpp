// mf_params.hpp -- kernel argument blocks shared by the host runtime and the
// kernels (plain structs passed by value as kernel arguments).
#pragma once

#include <stdint.h>

namespace mf {

// Conserved components per cell: E, Mx, My, Mz, and with the charge R (Sec. 2.1).
constexpr int kMaxComp = 5;

// Scheme constants of one sweep axis d (lambda = dt / dx_d).
template <typename T> struct AxisConst {
    T lam;        // dt / dx_d            (MUSTA predictor; alpha dt / dx_d as an ablation)
    T half_lam;   // dt / (2 dx_d)        (Hancock half step)
    T half_alam;  // alpha dt / (2 dx_d)  (Lax-Wendroff half step)
    T inv_2alam;  // dx_d / (2 alpha dt)  (Lax-Friedrichs viscosity)
    T inv_2dx;    // 1 / (2 dx_d)         (flux difference of G = 2 F)
};

// Grid of the learned seed's predictions: ln E in [kSeedLnLo, kSeedLnHi]
// (kSeedG0 points, E from 1e-4 to 1e4) by |M|/E in [0, 1] (kSeedG1 points).
constexpr int kSeedG0 = 1024, kSeedG1 = 513;
constexpr double kSeedLnLo = -9.210340371976184, kSeedLnHi = 9.210340371976184;

// Slots of the per-event device statistics block (uint64 each).
enum { ST_SMAX = 0, ST_FLOOR = 1, ST_BAD = 2, ST_ITERS = 3, ST_FALLBACK = 4, ST_WORDS = 8 };

// Runge-Kutta combine of the last axis sweep (Sec. 2.3):
//   RK_FIRST : out = u + dt L                                   (U1)
//   RK2_LAST : out = 1/2 ((u0 + u) + dt L)                      (U^{n+1}, RK2)
//   RK3_MID  : out = (3/4 u0 + 1/4 u) + 1/4 (dt L)              (U2, RK3)
//   RK3_LAST : out = (1/3 u0 + 2/3 u) + 2/3 (dt L)              (U^{n+1}, RK3)
enum { RK_FIRST = 0, RK2_LAST = 1, RK3_MID = 2, RK3_LAST = 3 };

// Modes of an axis sweep (fixed by the axis: x writes L, y adds to it, z
// finishes the stage).
enum { SW_WRITE = 0, SW_ACCUM = 1, SW_FINAL = 2 };

template <typename T> struct SweepArgs {
    // per component (4, or 5 with the charge R)
    const T* u[kMaxComp];    // stage input state (read with the stencil)
    T* L[kMaxComp];          // flux-divergence accumulator
    const T* u0[kMaxComp];   // Runge-Kutta base state U^n (SW_FINAL, kinds > RK_FIRST)
    T* out[kMaxComp];        // stage output (SW_FINAL)
    int64_t nlines;     // lines along the sweep axis
    int64_t stride_d;   // element stride along the sweep axis
    int64_t stride_f;   // stride of the fast line axis
    int64_t stride_s;   // stride of the slow line axis
    int32_t N;          // cells along the sweep axis
    int32_t n_fast;     // cells along the fast line axis
    int32_t seg;        // cells per thread along the sweep axis
    int32_t periodic;   // 1: periodic along the sweep axis, 0: outflow
    int32_t k;          // MUSTA stages
    int32_t kind;       // RK_* (SW_FINAL)
    int32_t want_smax;  // SW_FINAL: reduce the max characteristic speed of out
    int32_t axis_f;     // global axis of the fast line index
    int32_t axis_s;     // global axis of the slow line index
    AxisConst<T> ac;
    T dt;
    // moving point-jet source (SW_FINAL only)
    double jet_pos[3];    // jet position at the stage time (t_ptr == nullptr), else at t = 0
    const double* t_ptr;  // batched stepping: device event time; the stage time is *t_ptr + t_off
    double t_off;
    double jet_ve;        // v dE/dx
    double jet_v;         // v
    double jet_norm;      // (2 pi sigma^2)^(-3/2)
    double jet_inv2s2;    // 1 / (2 sigma^2)
    double origin[3];
    double dx[3];
    unsigned long long* stats;  // ST_WORDS per event
    // unsplit Hancock corrections (MF_FLAG_UNSPLIT_HANCOCK sweeps only): component c of
    // the extended cell (i, j, k), each in [-1, n], at dl[c * dl_n + ((k+1)(ny+2) + j+1)(nx+2) + i+1]
    const T* dl;
    int64_t dl_n;
    int64_t estride_d, estride_f, estride_s;  // extended strides along the sweep / fast / slow line axes
};

// Unsplit Hancock corrections over the extended grid (one thread per (x, y)
// column of it, marching zseg planes).
template <typename T> struct UnsplitArgs {
    const T* u[4];      // stage input state
    T* dl;              // 4 * dl_n corrections (layout as SweepArgs::dl)
    int64_t dl_n;
    int32_t n[3];
    int32_t periodic[3];
    int32_t zseg;       // extended z planes per thread (set by the launcher)
    T half_lam[3];      // dt / (2 dx_d)
    unsigned long long* stats;
};

template <typename T> struct C2PArgs {
    const T* U[kMaxComp];      // E, Mx, My, Mz (and R with the charge)
    T* prim[kMaxComp + 1];     // e, p, vx, vy, vz (and n with the charge)
    int32_t* iters;     // nullable
    int64_t n;
    unsigned long long* stats;
};

template <typename T> struct TotalsArgs {
    const T* U[kMaxComp];
    int64_t n;
    double* partial;    // kMaxComp per block
};


}  // namespace mf
