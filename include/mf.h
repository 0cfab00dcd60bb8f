/*
 * mf.h -- C ABI of the MI355X (gfx950) MUSTA-FORCE library for ideal
 * relativistic hydrodynamics.
 *
 * The library advances the conservation law dU/dt + dF/dx + dG/dy + dH/dz = 0
 * of Porter-Sobieraj et al., "A MUSTA-FORCE algorithm for solving partial
 * differential equations of relativistic hydrodynamics" (arXiv:1510.06340,
 * Sec. 2.1, conservation law and flux vectors), with U = (E, Mx, My, Mz),
 * by the dimensionally split scheme of Sec. 2.3-2.6: slope-limited MUSCL
 * reconstruction, a Hancock half step, a k-stage MUSTA predictor-corrector
 * with the FORCE centred flux on every interface, conserved-to-primitive
 * recovery and a TVD Runge-Kutta update.
 *
 * Conventions
 *  - Every call returns an int status: MF_OK (0) or a negative MF_ERR_*;
 *    mf_last_error() returns a message for the calling thread's last error.
 *  - State arrays are caller-owned device buffers (e.g. torch tensors), one
 *    array per conserved component, x fastest: cell (i, j, k) is element
 *    i + n[0] * (j + n[1] * k).  Their pointers are lent to the handle for
 *    its lifetime; the library never frees them.
 *  - Library-owned device scratch (Runge-Kutta stage states, the flux
 *    accumulator, statistics) is allocated by mf_grid_init and released by
 *    mf_grid_free.
 *  - Work is enqueued on the stream given to mf_grid_init (a hipStream_t;
 *    NULL = the default stream).  Calls that return host data synchronise
 *    that stream before returning.
 *  - Not thread-safe per handle: calls on one handle must not overlap.
 */
#ifndef MF_H
#define MF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ---------------------------------------------------- */
#define MF_OK 0
#define MF_ERR_ARG (-1)         /* invalid argument (sizes, pointers, codes) */
#define MF_ERR_NOMEM (-2)       /* device or host allocation failed */
#define MF_ERR_HIP (-3)         /* a HIP runtime call or kernel launch failed */
#define MF_ERR_STATE (-4)       /* call out of order (e.g. no EoS set) */
#define MF_ERR_UNPHYSICAL (-5)  /* MF_FLAG_STRICT and an unphysical state was met */
#define MF_ERR_CFL (-6)         /* MF_FLAG_STRICT and alpha * Courant number > 1 */

/* ---- codes ------------------------------------------------------------ */
enum mf_bc { MF_BC_OUTFLOW = 0, MF_BC_PERIODIC = 1 };
enum mf_dtype { MF_F64 = 0, MF_F32 = 1 };
enum mf_limiter {
    MF_LIM_NONE = 0,      /* central slope (U_{i+1} - U_{i-1}) / 2 */
    MF_LIM_MINMOD = 1,    /* Minbee  xi(r) = max(0, min(1, r)) */
    MF_LIM_SUPERBEE = 2,  /* xi(r) = max(0, min(2r, 1), min(r, 2)) */
    MF_LIM_MC = 3,        /* monotonised central xi(r) = max(0, min(2r, (1+r)/2, 2)) */
    MF_LIM_VANLEER = 4,   /* xi(r) = (r + |r|) / (1 + |r|) */
    MF_LIM_VANALBADA = 5  /* xi(r) = (r^2 + r) / (r^2 + 1) */
};
enum mf_eos_kind {
    MF_EOS_IDEAL = 0,  /* p = cs2 e */
    MF_EOS_TABLE = 1,  /* tabulated p(e), monotone cubic */
    MF_EOS_GAMMA = 2   /* ideal gas p = (gamma - 1) max(e - n, 0), n the rest-frame charge
                          density (needs MF_FLAG_CHARGE) */
};
enum mf_c2p_mode {
    MF_C2P_PLAIN = 0,     /* bracketed Newton from the bracket midpoint (table) / closed form (ideal) */
    MF_C2P_SEEDED = 1,    /* table EoS: guess from the learned seed network, evaluated on the matrix cores */
    MF_C2P_CONFORMAL = 2  /* table EoS: guess from the p = e/3 closed form (a baseline for the seed) */
};

#define MF_FLAG_STRICT 1u  /* mf_step fails on unphysical states or alpha*Courant > 1 */
#define MF_FLAG_PREDICTOR_ALPHA 2u  /* ablation of the MUSTA predictor coefficient: alpha dt/dx
                                       instead of dt/dx as printed in Sec. 2.4 (the FORCE
                                       fluxes use alpha dt/dx either way) */
#define MF_FLAG_UNSPLIT_HANCOCK 4u  /* ablation of the multi-dimensional Hancock half step
                                       (Sec. 2.4 MUSCL-Hancock): one correction per cell,
                                       sum_d (dt/2dx_d)(F_d(U^{L,d}) - F_d(U^{R,d})) over the three
                                       axes, added to the faces of every sweep, instead of each
                                       sweep's own axis term.  mf_step only (mf_batch_step
                                       returns MF_ERR_ARG); the library allocates
                                       4 (n0+2)(n1+2)(n2+2) elements per event for it */

#define MF_FLAG_CHARGE 8u  /* a fifth conserved component, the charge R = n gamma of Sec. 2.1
                              (flux R v_d; n = R sqrt(1 - v^2), Sec. 2.6): U_dev holds 5
                              pointers per event (E, Mx, My, Mz, R).  All events of a handle
                              carry it or none does; FP64 only; with MF_EOS_IDEAL (a passive
                              charge) or MF_EOS_GAMMA, through mf_step (not mf_batch_step,
                              the jet source or MF_FLAG_UNSPLIT_HANCOCK: MF_ERR_ARG) */

typedef struct mf_grid_s* mf_grid_t;

/* One event (one grid).  Sec. 2.4: alpha = 3 in three dimensions. */
typedef struct {
    int32_t n[3];       /* cells along x, y, z (each >= 1) */
    double dx[3];       /* cell sizes (> 0) */
    double origin[3];   /* lower box corner; cell centres at origin + (i + 1/2) dx */
    int32_t bc[3];      /* mf_bc per axis */
    int32_t dtype;      /* mf_dtype of the state arrays and of the arithmetic */
    int32_t limiter;    /* mf_limiter */
    int32_t musta_k;    /* MUSTA stages k >= 1 (k = 1 is plain FORCE) */
    int32_t rk_order;   /* 2 or 3 (Sec. 2.3) */
    double alpha;       /* FORCE coefficient (> 0) */
    uint32_t flags;     /* MF_FLAG_* */
} mf_grid_desc;

/* Per-event statistics of one mf_step / mf_batch_step call. */
typedef struct {
    double t;             /* event time after the call */
    int64_t steps;        /* steps taken by this event since mf_grid_init */
    double smax;          /* max |characteristic speed| over cells, axes and end-of-step states */
    double courant;       /* smax * dt / min(dx) */
    double totals[4];     /* sum over cells of (E, Mx, My, Mz) * dV of the final state */
    int64_t n_floor;      /* con2prim calls whose |M| was clamped to (1 - 1e-12) E */
    int64_t n_bad;        /* con2prim calls with E <= 0 or non-finite input */
    int64_t newton_iters; /* Newton / bisection iterations of the table EoS */
    int64_t n_fallback;   /* seeded con2prim solves whose guess lay outside the bracket (started at its midpoint) */
} mf_stats;

/* Optional learned con2prim seed for MF_EOS_TABLE: a 2 -> H -> H -> 1 tanh
 * MLP (H = 64) on x = ((ln E - in_shift[0]) * in_scale[0], (|M|/E - in_shift[1]) * in_scale[1])
 * predicting z = out_scale * y + out_shift (ln e, or the bracket fraction, by
 * `output`).  Weights row-major FP32 host arrays, copied by mf_set_eos and
 * rounded to bfloat16 on the device.  The sweeps read the network's
 * predictions from a (ln E, |M|/E) grid the network fills once per
 * mf_set_eos; mf_con2prim(MF_C2P_SEEDED) evaluates it per state.  The guess
 * starts the same safeguarded Newton solve as the plain one (Sec. 2.6 inverse)
 * if it lies strictly inside the bracket [E - |M|^2/E, E], else the solve
 * starts at the bracket midpoint; results equal the plain solve's to the
 * solver's tolerance either way. */
typedef struct {
    int32_t hidden;      /* H (multiple of 16, <= 256) */
    const float* w1;     /* H x 2 */
    const float* b1;     /* H */
    const float* w2;     /* H x H */
    const float* b2;     /* H */
    const float* w3;     /* 1 x H */
    float b3;
    float in_shift[2], in_scale[2];
    float out_shift, out_scale;
    int32_t output;      /* 0: z = ln e;
                            1: z = the bracket fraction (E - e) E / |M|^2, so e = E - z |M|^2 / E */
} mf_surrogate;

/* Create a handle for n_events independent grids (Sec. 2.1 problem statement,
 * one descriptor per event).  U_dev holds 4 device pointers per event
 * (E, Mx, My, Mz, each n[0]*n[1]*n[2] elements of the event's dtype), or 5
 * (E, Mx, My, Mz, R) with MF_FLAG_CHARGE.
 * stream: hipStream_t or NULL.  Errors: MF_ERR_ARG (n < 1, dx <= 0, k < 1,
 * rk not 2/3, alpha <= 0, unknown codes, NULL pointers), MF_ERR_NOMEM, MF_ERR_HIP. */
int mf_grid_init(mf_grid_t* out, const mf_grid_desc* descs, int32_t n_events,
                 void* const* U_dev, void* stream);

/* Equation of state (Sec. 2.1, closure p = p(e, n)).
 * MF_EOS_IDEAL: p = cs2 * e with 0 < cs2 < 1; the table arguments are ignored.
 * MF_EOS_GAMMA: the ideal gas p = (gamma - 1) max(e - n, 0) with the adiabatic
 * index gamma in [1, 2] passed as cs2 (gamma = 1: pressureless dust); needs
 * MF_FLAG_CHARGE.  con2prim solves the fixed point of Sec. 2.6 for p by
 * safeguarded Newton; cold gas (p = 0) is exact.
 * MF_EOS_TABLE: n_tab >= 3 host nodes (e_tab strictly increasing, > 0;
 * p_tab non-decreasing, >= 0, p < e) interpolated by a monotone piecewise
 * cubic; below e_tab[0] p = p_tab[0] e / e_tab[0], above the last node linear
 * with the end slope.  Fast interval lookup assumes log-uniform nodes and
 * falls back to bisection otherwise.  s (nullable) attaches the learned seed.
 * Host arrays are copied.  Errors: MF_ERR_ARG (also MF_EOS_TABLE with the
 * charge, MF_EOS_GAMMA without it). */
int mf_set_eos(mf_grid_t g, int32_t kind, double cs2, const double* e_tab,
               const double* p_tab, int32_t n_tab, const mf_surrogate* s);

/* Moving point-jet source for one event: adds to dE/dt and dMx/dt
 * S = v dEdx G_sigma(x - x0 - v t e_x) (1, v, 0, 0), G_sigma the normalised
 * 3-D Gaussian of width sigma sampled at cell centres.  0 < v < 1, sigma > 0;
 * dEdx = 0 switches it off. */
int mf_set_source_jet(mf_grid_t g, int32_t event, const double x0[3], double v,
                      double dEdx, double sigma);

/* Set an event's time t (used by the source term; resume from a checkpoint). */
int mf_set_time(mf_grid_t g, int32_t event, double t, int64_t steps);

/* Advance every event by nsteps Runge-Kutta steps of size dt (Sec. 2.3), one
 * event after another.  st (nullable) receives n_events entries; passing it
 * synchronises the stream.  Unphysical states are clamped and counted; with
 * MF_FLAG_STRICT they make the call return MF_ERR_UNPHYSICAL, and
 * alpha * Courant > 1 returns MF_ERR_CFL (the state is advanced either way).
 * Errors: MF_ERR_STATE (no EoS), MF_ERR_ARG (dt <= 0, nsteps < 0), MF_ERR_HIP. */
int mf_step(mf_grid_t g, double dt, int32_t nsteps, mf_stats* st);

/* Advance all events together, event i by nsteps steps of size dt[i] (host
 * array): each Runge-Kutta stage sweep is one persistent launch over a tile
 * queue spanning every event, and a step is replayed from a captured HIP
 * graph.  Results equal mf_step's per event.  st as in mf_step. */
int mf_batch_step(mf_grid_t g, const double* dt, int32_t nsteps, mf_stats* st);

/* Conserved -> primitive recovery (Sec. 2.6) of n states with the handle's
 * EoS and dtype: U = 4 device arrays (E, Mx, My, Mz), prim = 5 device arrays
 * (e, p, vx, vy, vz); with MF_FLAG_CHARGE U = 5 (R last) and prim = 6 (the
 * rest-frame charge density n = R sqrt(1 - v^2) last).  iters_dev (nullable, int32 device array of n) receives
 * the root-finder iterations per state (0 for the closed form).  mode:
 * MF_C2P_PLAIN (midpoint start, whether or not a seed is installed),
 * MF_C2P_SEEDED (needs a surrogate) or MF_C2P_CONFORMAL.  Asynchronous. */
int mf_con2prim(mf_grid_t g, const void* const U[], void* const prim[], int64_t n,
                int32_t* iters_dev, int32_t mode);

/* Counters of the last mf_con2prim call: out = (clamped |M|, bad states,
 * root-finder iterations, seeded guesses outside the bracket).  Synchronous. */
int mf_con2prim_stats(mf_grid_t g, int64_t out[4]);

/* ---- the seed network's training kernels (BF16 matrix cores, FP32 accumulation)
 * Parameters: MF_MLP_PARAMS FP32 values in device memory, laid out
 * W1[64][2], b1[64], W2[64][64], b2[64], w3[64], b3 (row-major).  Inputs X are
 * n x 2 FP32 (row-major), targets and outputs n FP32; all device pointers,
 * asynchronous on 'stream' (hipStream_t or NULL). */
#define MF_MLP_HIDDEN 64
#define MF_MLP_PARAMS 4417
/* Scratch (in floats) that mf_mlp_grad needs for n samples. */
int64_t mf_mlp_workspace(int64_t n);
/* y = MLP(X). */
int mf_mlp_forward(const float* params, const float* X, int64_t n, float* y, void* stream);
/* Gradient of mean((MLP(X) - t)^2) into grad[MF_MLP_PARAMS]; the loss into
 * *loss (device, nullable).  work: mf_mlp_workspace(n) floats. */
int mf_mlp_grad(const float* params, const float* X, const float* t, int64_t n, float* grad, float* loss,
                float* work, int64_t work_floats, void* stream);
/* For callers that cannot allocate device memory (code under HIP graph capture,
 * tight training or serving loops, harnesses that forbid allocation): the same
 * gradient as mf_mlp_grad, with its partial gradients (one per block of 64
 * samples) kept in a library-owned static device array instead of a caller
 * workspace.  The array holds the partials of up to MF_MLP_NOALLOC_MAX_N
 * samples (1.1 MB); each GPU
 * the library runs on holds its own copy until the process ends.  n must lie
 * in [1, MF_MLP_NOALLOC_MAX_N] (else MF_ERR_ARG).  The call runs on the current
 * device, and stream must belong to it.  It allocates nothing: no hipMalloc,
 * hipFree or allocating library routine.  Every call on one GPU shares that
 * GPU's array, and each call rewrites every partial it reads, so nothing is
 * carried from one call to the next; calls that overlap on one GPU (two
 * streams, or two host threads) race on the array and must be serialised by
 * the caller.  Other arguments and errors as in mf_mlp_grad. */
#define MF_MLP_NOALLOC_MAX_N 16384
int mf_mlp_grad_noalloc(const float* params, const float* X, const float* t, int64_t n, float* grad, float* loss,
                        void* stream);
/* One Adam step (step >= 1) on params with moments m, v (MF_MLP_PARAMS each). */
int mf_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t step, float lr, float beta1,
                float beta2, float eps, void* stream);

/* Sums of (E, Mx, My, Mz) * dV over one event's cells (deterministic order),
 * and of R * dV as out[4] with MF_FLAG_CHARGE (out then holds 5 doubles).
 * Synchronous. */
int mf_totals(mf_grid_t g, int32_t event, double* out);

/* Per-step kernel shape (0 = automatic): seg[0] = chunks of 64 row items per
 * wavefront of the x sweep, seg[1], seg[2] = cells per thread along y and z;
 * block = threads per block (64, 128 or 256).  Used by the autotuner. */
int mf_set_tuning(mf_grid_t g, const int32_t seg[3], int32_t block);

/* Kernel timing: with enable != 0 every axis-sweep launch is bracketed by
 * HIP events on the handle's stream.  mf_get_profile synchronises the stream
 * and returns, per sweep axis (x, y, z), the summed kernel time in
 * milliseconds and the number of launches since profiling was enabled or
 * last read; then it resets the counts. */
int mf_set_profiling(mf_grid_t g, int32_t enable);
int mf_get_profile(mf_grid_t g, double ms[3], int64_t launches[3]);

/* Release the handle and its scratch (the caller's state arrays are untouched). */
int mf_grid_free(mf_grid_t g);

/* Message of the calling thread's last error ("" if none). */
const char* mf_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* MF_H */
