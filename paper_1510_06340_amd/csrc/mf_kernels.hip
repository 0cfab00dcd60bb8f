// mf_kernels.hip -- gfx950 kernels of the MUSTA-FORCE step.
//
// y and z sweeps (k_sweep): one thread owns a segment of one grid line along
// the sweep axis and marches along it with a three-cell register window (and
// the next cell loaded one step ahead), so
// each cell's reconstruction + Hancock half step and each interface's
// MUSTA-FORCE flux is computed once (plus two cells and one interface of
// overlap per segment).  Lanes of a wavefront own neighbouring x cells, so
// every load and store is one contiguous 512-byte (FP64) row.
// x sweep (k_sweep_x): lanes lie along x over a stream of row items and pass
// face states and fluxes to their neighbours by DPP lane shifts (across
// chunks through LDS).
// The three sweeps of a Runge-Kutta stage accumulate L = ((Lx + Ly) + Lz) in
// a library-owned array; the z sweep also adds the source term, applies the
// Runge-Kutta combine and (last stage) reduces the max characteristic speed.
// k_batch_sweep runs the same per-thread code for many events from one
// persistent launch over a tile queue.
#include <hip/hip_runtime.h>
#include <type_traits>

#include <algorithm>

#include "mf_device.hpp"
#include "mf_index.hpp"
#include "mf_kernels.hpp"

namespace mf {

template <typename T>
__device__ __forceinline__ void load4(const T* const u[], int64_t i, T w[4])
{
    w[0] = u[0][i]; w[1] = u[1][i]; w[2] = u[2][i]; w[3] = u[3][i];
}

template <typename T>
__device__ __forceinline__ void copy4(const T a[4], T b[4])
{
    b[0] = a[0]; b[1] = a[1]; b[2] = a[2]; b[3] = a[3];
}

// NC conserved components (4, or 5 with the charge R) of cell i.
template <int NC, typename T>
__device__ __forceinline__ void loadn(const T* const u[], int64_t i, T w[])
{
#pragma unroll
    for (int c = 0; c < NC; c++) w[c] = u[c][i];
}

template <int NC, typename T>
__device__ __forceinline__ void copyn(const T a[], T b[])
{
#pragma unroll
    for (int c = 0; c < NC; c++) b[c] = a[c];
}

__device__ __forceinline__ void add_counts(Counts& a, const Counts& b)
{
    a.floor_ += b.floor_;
    a.bad += b.bad;
    a.iters += b.iters;
    a.fallback += b.fallback;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Flush per-thread counters and the speed maximum: one atomic per wavefront.
template <typename T>
__device__ __forceinline__ void flush_stats(unsigned long long* st, const Counts& cnt, T smax,
                                            bool want_smax)
{
    const uint32_t f = wave_sum(cnt.floor_);
    const uint32_t b = wave_sum(cnt.bad);
    const uint32_t it = wave_sum(cnt.iters);
    const uint32_t fb = wave_sum(cnt.fallback);
    double sm = 0.0;
    if (want_smax) sm = (double)wave_max(smax);
    if ((threadIdx.x & 63) == 0) {
        if (f) atomicAdd(&st[ST_FLOOR], (unsigned long long)f);
        if (b) atomicAdd(&st[ST_BAD], (unsigned long long)b);
        if (it) atomicAdd(&st[ST_ITERS], (unsigned long long)it);
        if (fb) atomicAdd(&st[ST_FALLBACK], (unsigned long long)fb);
        if (want_smax && sm > 0.0) atomicMax(&st[ST_SMAX], (unsigned long long)__double_as_longlong(sm));
    }
}


// What the sweep along axis D does with its flux divergence: the x sweep
// writes L, the y sweep adds to it, the z sweep finishes the stage.  A
// compile-time constant, so each kernel holds (and keeps registers for) only
// the arrays its mode uses.
template <int D>
constexpr int sweep_mode()
{
    return D == 0 ? SW_WRITE : (D == 1 ? SW_ACCUM : SW_FINAL);
}

// Output of one cell of an axis sweep: write or accumulate L, or (last axis)
// add the source, apply the Runge-Kutta combine and track the max speed.
// uin = U[cell] of the stage input, Lp = L so far, ub = RK base state,
// SE = energy source of the cell (jet only; jet_source below).
template <typename T, bool JET, int MODE, int NC = 4, class Eos>
__device__ __forceinline__ void emit_cell(const SweepArgs<T>& a, const Eos& eos, int64_t ij, const T uin[],
                                          const T Ld[], const T Lp[], const T ub[], T SE, T& smax)
{
    if constexpr (MODE == SW_WRITE) {
#pragma unroll
        for (int c = 0; c < NC; c++) a.L[c][ij] = Ld[c];
        return;
    }
    if constexpr (MODE == SW_ACCUM) {
#pragma unroll
        for (int c = 0; c < NC; c++) a.L[c][ij] = Lp[c] + Ld[c];
        return;
    }
    T Lt[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) Lt[c] = Lp[c] + Ld[c];
    if constexpr (JET) {
        Lt[0] = Lt[0] + SE;
        Lt[1] = Lt[1] + T(a.jet_v) * SE;
    }
    T o[NC];
    const T dt = a.dt;
    if (a.kind == RK_FIRST) {
#pragma unroll
        for (int c = 0; c < NC; c++) o[c] = uin[c] + dt * Lt[c];
    } else if (a.kind == RK2_LAST) {
#pragma unroll
        for (int c = 0; c < NC; c++) o[c] = T(0.5) * ((ub[c] + uin[c]) + dt * Lt[c]);
    } else if (a.kind == RK3_MID) {
#pragma unroll
        for (int c = 0; c < NC; c++) o[c] = (T(0.75) * ub[c] + T(0.25) * uin[c]) + T(0.25) * (dt * Lt[c]);
    } else {
        const T third = T(1.0 / 3.0), two3 = T(2.0 / 3.0);
#pragma unroll
        for (int c = 0; c < NC; c++) o[c] = (third * ub[c] + two3 * uin[c]) + two3 * (dt * Lt[c]);
    }
#pragma unroll
    for (int c = 0; c < NC; c++) a.out[c][ij] = o[c];
    if (a.want_smax) {
        T e, p, v[3], cs2;
        Counts cs;
        eos.prim(o, e, p, v, cs2, cs);
        smax = fmax(smax, max_speed(v, cs2));
    }
}

// Jet energy source S_E = v dE/dx G_sigma(x - x_jet(t)) at a cell centre at
// squared distance r2 from the jet (the momentum source is v S_E).  Where the
// exponent is below -746 the exponential is exactly 0 in FP64 (and FP32), so
// wavefronts far from the jet skip it.
template <typename T>
__device__ __forceinline__ T jet_source(const SweepArgs<T>& a, double r2)
{
    const double arg = r2 * a.jet_inv2s2;
    const bool near = arg < 746.0;
    T SE = T(0);
    if (__any(near)) {
        if (near) SE = T(a.jet_ve) * (T(a.jet_norm) * exp(-T(arg)));
    }
    return SE;
}

// Lane i receives v from lane i-1; lane 0 receives 'carry' (DPP wave shift right).
__device__ __forceinline__ double shift_up1(double v, double carry)
{
    const long long x = __double_as_longlong(v);
    const long long c = __double_as_longlong(carry);
    const int lo = __builtin_amdgcn_update_dpp((int)c, (int)x, 0x138, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp((int)(c >> 32), (int)(x >> 32), 0x138, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ __forceinline__ float shift_up1(float v, float carry)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(carry), __float_as_int(v), 0x138, 0xf, 0xf,
                                                      false));
}

// One thread's segment [s0, s0 + seg) of grid line 'line' along axis D.
// UNSPLIT (the MF_FLAG_UNSPLIT_HANCOCK ablation): the faces take the cell's
// three-axis correction from a.dl instead of this axis' Hancock term.
// NC: conserved components (4, or 5 with the charge R).
template <typename T, int D, int LIM, class Eos, bool JET, bool UNSPLIT = false, int NC = 4>
__device__ __forceinline__ void sweep_line(const SweepArgs<T>& a, const Eos& eos, int64_t line, int s0,
                                           Counts& cnt, T& smax)
{
    const int N = a.N;
    if (!(line < a.nlines && s0 < N)) return;
    const int s1 = min(s0 + a.seg, N);
    const int64_t i_f = line % a.n_fast;
    const int64_t i_s = line / a.n_fast;
    const int64_t base = i_f * a.stride_f + i_s * a.stride_s;
    // this line's cells in the extended grid of the unsplit corrections
    const int64_t ebase = UNSPLIT ? (i_f + 1) * a.estride_f + (i_s + 1) * a.estride_s : 0;
    const int64_t sd = a.stride_d;
    auto cell = [&](int j) -> int64_t { return base + (int64_t)ghost(j, N, a.periodic) * sd; };

    // The march starts two cells early: iteration j reconstructs cell j+1
    // and (from j = s0-1 on) solves interface j+1/2; cells are written
    // from j = s0 on.  Warm-up and body share one instance of the code,
    // so results do not depend on the segmentation.
    // jet source (z sweep): squared distance from the jet in the (x, y) plane of this line
    double jet_dxy2 = 0.0;
    if constexpr (JET && D == 2) {  // the line index runs over (x, y)
        const double xj = a.jet_pos[0] + (a.t_ptr ? a.jet_v * (*a.t_ptr + a.t_off) : 0.0);
        const double x = a.origin[0] + (i_f + 0.5) * a.dx[0] - xj;
        const double y = a.origin[1] + (i_s + 0.5) * a.dx[1] - a.jet_pos[1];
        jet_dxy2 = x * x + y * y;
    }

    static_assert(NC == 4 || !UNSPLIT, "the unsplit ablation carries four components");
    T w0[NC], w1[NC], w2[NC], wn[NC];
    T ULt[NC], URt[NC], URp[NC], Fp[NC], Fn[NC];
    loadn<NC>(a.u, cell(s0 - 2), w1);
    loadn<NC>(a.u, cell(s0 - 1), w2);
    loadn<NC>(a.u, cell(s0), wn);
    for (int j = s0 - 2; j < s1; j++) {
        copyn<NC>(w1, w0);
        copyn<NC>(w2, w1);
        copyn<NC>(wn, w2);
        // cell j+3 is loaded one step ahead (its latency hides behind this
        // step); march_ahead keeps the last iteration's load, whose value is
        // never used, inside the line
        loadn<NC>(a.u, cell(march_ahead(j, N)), wn);
        const int64_t ij = base + (int64_t)j * sd;
        const bool body = j >= s0;
        constexpr int MODE = sweep_mode<D>();
        // With Eos::kLoadLAhead the L so far (and, in the z sweep, the stage's
        // u0) is loaded before the cell's work, whose latency hides it; the
        // jet's z sweep has no registers to spare for it
        constexpr bool early_L =
            Eos::kLoadLAhead && (MODE == SW_ACCUM || (MODE == SW_FINAL && !JET));
        T Lp[NC], ub[NC];
#pragma unroll
        for (int c = 0; c < NC; c++) {
            Lp[c] = T(0);
            ub[c] = T(0);
        }
        if constexpr (early_L) {
            if (body) {
                loadn<NC>((const T* const*)a.L, ij, Lp);
                if constexpr (MODE == SW_FINAL) {
                    if (a.kind != RK_FIRST) loadn<NC>(a.u0, ij, ub);
                }
            }
        }
        // the jet source of cell j, evaluated here where few values are live
        T SE = T(0);
        if constexpr (JET && D == 2) {
            if (body) {
                const double z = a.origin[2] + (j + 0.5) * a.dx[2] - a.jet_pos[2];
                SE = jet_source(a, jet_dxy2 + z * z);
            }
        }

        // cell j+1; counted once over all segments of the line (cells -1..N)
        const int c1 = j + 1;
        cnt.w = (c1 == s0 - 1 ? s0 == 0 : (c1 < s1 || c1 == N)) ? 1u : 0u;
        if constexpr (UNSPLIT) {
            // cell j+1 in [s0-1, s1], extended coordinate j+2 in [0, N+1].  Loading
            // it a step ahead like the states was tried: the extra registers
            // made the z sweep spill, and it ran slower.
            T d[4];
            load_dl(a.dl + ebase + (int64_t)(j + 2) * a.estride_d, a.dl_n, d);
            unsplit_faces<LIM>(w0, w1, w2, d, ULt, URt);
        } else {
            hancock<D, LIM, true, NC>(w0, w1, w2, a.ac.half_lam, ULt, URt, eos, cnt);
        }
        if (j == s0 - 2) {
            copyn<NC>(URt, URp);
            continue;
        }
        // interface j + 1/2; counted once over all segments (interfaces -1/2..N-1/2)
        cnt.w = (body || s0 == 0) ? 1u : 0u;
        musta<D, true, NC>(URp, ULt, a.k, a.ac, Fn, eos, cnt);
        copyn<NC>(URt, URp);
        if (!body) {
            copyn<NC>(Fn, Fp);
            continue;
        }

        T Ld[NC];
        if constexpr (MODE != SW_WRITE && !early_L) loadn<NC>((const T* const*)a.L, ij, Lp);
        if constexpr (MODE == SW_FINAL && !early_L) {
            if (a.kind != RK_FIRST) loadn<NC>(a.u0, ij, ub);
        }
#pragma unroll
        for (int c = 0; c < NC; c++) Ld[c] = -(Fn[c] - Fp[c]) * a.ac.inv_2dx;   // Fn, Fp: G = 2 F
        emit_cell<T, JET, MODE, NC>(a, eos, ij, w0, Ld, Lp, ub, SE, smax);
        copyn<NC>(Fn, Fp);
    }
}

// Waves per SIMD the register budget is sized for.  The jet source adds a
// few live values to the z sweep, which at 4 waves (3 with the table EoS)
// would spill: it gets one wavefront fewer.
template <class Eos, bool JET>
constexpr int sweep_waves()
{
    return JET && Eos::kWaves > 2 ? Eos::kWaves - 1 : Eos::kWaves;
}

template <typename T, int D, int LIM, class Eos, bool JET, bool UNSPLIT = false, int NC = 4>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sweep_waves<Eos, JET>()))) void k_sweep(SweepArgs<T> a, Eos eos)
{
    __shared__ double eos_cache[Eos::kCacheDoubles];
    eos.bind_cache(eos_cache);
    const int64_t line = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    Counts cnt;
    T smax = T(0);
    sweep_line<T, D, LIM, Eos, JET, UNSPLIT, NC>(a, eos, line, (int)blockIdx.y * a.seg, cnt, smax);
    flush_stats(a.stats, cnt, smax, sweep_mode<D>() == SW_FINAL && a.want_smax);
}

// ---------------------------------------------------------------------------
// x sweep with lanes along x.  The rows of the grid are read as one stream of
// items (row, x), x = -1..N (the cells whose faces feed the N+1 interfaces of
// the row).  A wavefront takes 64 consecutive items per chunk: each lane
// reconstructs its cell, receives its left neighbour's right face state by a
// DPP lane shift (lane 0 from the previous chunk's lane 63, through LDS), solves the
// interface between them, receives the left neighbour's flux the same way and
// writes L for the cell on its left.  All loads and stores are coalesced.
// A wavefront owns items [s, s + 64 * seg) and starts two items early.
// ---------------------------------------------------------------------------
// The x sweep evaluates the face fluxes one after the other for p = c e (its
// five wavefronts per SIMD hide the latency); with the table EoS it pairs the
// lookups (flux2), which since the piece cache moved to LDS still fits four
// wavefronts per SIMD, and with the ideal gas it takes the pairs so that the
// pressure iterations start from the pair's neighbour.
template <class Eos>
constexpr bool kPairX = std::is_same<Eos, EosTable>::value || std::is_same<Eos, EosGamma>::value;

// Wavefront 'wave' of the x sweep: items [wave * 64 * seg, ...) of the row stream.
// carry: this wavefront's 2 NC LDS slots, through which lane 63 hands its right
// face state and flux to lane 0 of the next chunk (LDS traffic instead of
// lane reads into scalar registers and moves back).
template <typename T, int LIM, class Eos, bool UNSPLIT = false, int NC = 4>
__device__ __forceinline__ void sweep_x_wave(const SweepArgs<T>& a, const Eos& eos, int64_t wave, int lane,
                                             T* carry, Counts& cnt, T& smax)
{
    const int N = a.N;
    const int64_t P = (int64_t)N + 2;
    const int64_t total = a.nlines * P;
    const int64_t s = wave * 64 * (int64_t)a.seg;
    if (s < total) {
        const int64_t e = min(s + 64 * (int64_t)a.seg, total);
        int64_t it = s - 2 + lane;
        int64_t row = 0;
        int x = 0;
        if (it >= 0) {
            x_item(it, N, row, x);
        } else {
            x = (int)(it + P) - 1;  // before the first row: never valid
            row = -1;
        }
        if (lane == 63) {
#pragma unroll
            for (int c = 0; c < 2 * NC; c++) carry[c] = T(0);
        }
        __builtin_amdgcn_wave_barrier();
        for (int64_t c0 = s - 2; c0 < e; c0 += 64) {
            it = c0 + lane;
            const bool valid = (it >= 0) & (it < e);
            const int64_t base = (valid ? row : 0) * (int64_t)N;
            const int xc = valid ? x : 0;
            static_assert(NC == 4 || !UNSPLIT, "the unsplit ablation carries four components");
            T w0[NC], w1[NC], w2[NC];
            // chunks away from row edges (most of them) need no ghost mapping:
            // the neighbours are the adjacent elements
            const uint64_t edge = lanes_where(!valid) | lanes_where(xc < 1) | lanes_where(xc > N - 2);
            if (edge == 0) {
                const int64_t ic = base + xc;
                loadn<NC>(a.u, ic - 1, w0);
                loadn<NC>(a.u, ic, w1);
                loadn<NC>(a.u, ic + 1, w2);
            } else {
                loadn<NC>(a.u, base + ghost(xc - 1, N, a.periodic), w0);
                loadn<NC>(a.u, base + ghost(xc, N, a.periodic), w1);
                loadn<NC>(a.u, base + ghost(xc + 1, N, a.periodic), w2);
            }
            T ULt[NC], URt[NC];
            cnt.w = (valid & (it >= s)) ? 1u : 0u;
            if constexpr (UNSPLIT) {
                // the lane's cell xc in [-1, N] of row (y, z) = (r % ny, r / ny), r in [0, ny nz)
                const int64_t r = valid ? row : 0;
                const int64_t e = (int64_t)(xc + 1) * a.estride_d + (r % a.n_fast + 1) * a.estride_f +
                                  (r / a.n_fast + 1) * a.estride_s;
                T d[4];
                load_dl(a.dl + e, a.dl_n, d);
                unsplit_faces<LIM>(w0, w1, w2, d, ULt, URt);
            } else {
                hancock<0, LIM, kPairX<Eos>, NC>(w0, w1, w2, a.ac.half_lam, ULt, URt, eos, cnt);
            }
            T URl[NC];
#pragma unroll
            for (int c = 0; c < NC; c++) URl[c] = shift_up1(URt[c], carry[c]);
            T F[NC];
#pragma unroll
            for (int c = 0; c < NC; c++) F[c] = T(0);
            if (valid & (x >= 0) & (it >= s - 1)) {   // interface x - 1/2
                cnt.w = (it >= s) ? 1u : 0u;
                musta<0, kPairX<Eos>, NC>(URl, ULt, a.k, a.ac, F, eos, cnt);
            }
            T Fl[NC];
#pragma unroll
            for (int c = 0; c < NC; c++) Fl[c] = shift_up1(F[c], carry[NC + c]);
            if (valid & (x >= 1) & (it >= s)) {   // cell x - 1
                const int64_t ij = base + (x - 1);
                T Ld[NC], Lp[NC], ub[NC];
#pragma unroll
                for (int c = 0; c < NC; c++) {
                    Ld[c] = -(F[c] - Fl[c]) * a.ac.inv_2dx;   // F, Fl: G = 2 F
                    Lp[c] = T(0);
                    ub[c] = T(0);
                }
                emit_cell<T, false, SW_WRITE, NC>(a, eos, ij, w0, Ld, Lp, ub, T(0), smax);
            }
            __builtin_amdgcn_wave_barrier();   // every lane has read the carry
            if (lane == 63) {
#pragma unroll
                for (int c = 0; c < NC; c++) {
                    carry[c] = URt[c];
                    carry[NC + c] = F[c];
                }
            }
            __builtin_amdgcn_wave_barrier();
            x += 64;
            while (x > N) {
                x -= (int)P;
                row++;
            }
        }
    }
}

template <typename T, int LIM, class Eos, bool UNSPLIT = false, int NC = 4>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(Eos::kWaves))) void k_sweep_x(SweepArgs<T> a, Eos eos)
{
    __shared__ T carry[256 / 64][2 * NC];
    __shared__ double eos_cache[Eos::kCacheDoubles];
    eos.bind_cache(eos_cache);
    Counts cnt;
    T smax = T(0);
    sweep_x_wave<T, LIM, Eos, UNSPLIT, NC>(a, eos, ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6,
                                           threadIdx.x & 63, carry[threadIdx.x >> 6], cnt, smax);
    flush_stats(a.stats, cnt, smax, false);   // the x sweep writes L only
}


// ---------------------------------------------------------------------------
// Unsplit Hancock corrections (the MF_FLAG_UNSPLIT_HANCOCK ablation), one
// thread per cell of the grid extended by one ghost cell per side:
//   dl = sum_d (dt / 2dx_d) (F_d(U^{L,d}) - F_d(U^{R,d})),
// U^{L,d}, U^{R,d} the limited faces along axis d, the state outside the grid
// from each axis' boundary condition (ghost indices in [-2, n+1]).
// ---------------------------------------------------------------------------
// The seven stencil states are loaded before any flux work so that their
// latencies overlap; neighbours along axis d differ from the centre in that
// coordinate only.
template <int D, int LIM, typename T, class Eos>
__device__ __forceinline__ void unsplit_axis(const UnsplitArgs<T>& a, const Eos& eos, const T wm[4], const T w0[4],
                                             const T wp[4], T delta[4], Counts& cnt)
{
    T UL[4], UR[4], FL[4], FR[4];
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const T hs = half_slope<LIM>(w0[c] - wm[c], wp[c] - w0[c]);
        UL[c] = w0[c] - hs;
        UR[c] = w0[c] + hs;
    }
    eos.template flux<D>(UL, FL, cnt);
    eos.template flux<D>(UR, FR, cnt);
#pragma unroll
    for (int c = 0; c < 4; c++) delta[c] = delta[c] + a.half_lam[D] * (FL[c] - FR[c]);
}

// One thread per (x, y) column of the extended grid, marching the extended z
// planes [z0, z1): the z-1, z and z+1 states stay in registers, so each plane
// loads its own cell and its four x/y neighbours.  Blocks are dealt to the 8
// XCDs round-robin; chunk c of 256 columns goes to block 8 (c % per) + c / per,
// so consecutive chunks (neighbouring rows, whose y neighbours they share)
// run on one XCD and meet in its L2.  gridDim.x is a multiple of 8.
template <typename T, int LIM, class Eos>
__global__ __launch_bounds__(256) void k_unsplit_delta(UnsplitArgs<T> a, Eos eos)
{
    __shared__ double eos_cache[Eos::kCacheDoubles];
    eos.bind_cache(eos_cache);
    const int64_t per = gridDim.x / 8;
    const int64_t chunk = (int64_t)(blockIdx.x % 8) * per + blockIdx.x / 8;
    const int64_t col = chunk * blockDim.x + threadIdx.x;
    const int64_t ex = a.n[0] + 2, ey = a.n[1] + 2;
    const int ez = a.n[2] + 2;
    const int z0 = (int)blockIdx.y * a.zseg;
    Counts cnt;
    if (col < ex * ey && z0 < ez) {
        const int z1 = min(z0 + a.zseg, ez);
        const int64_t row = col / ex;
        const int q0 = (int)(col - row * ex) - 1, q1 = (int)row - 1;
        const int64_t sy = a.n[0], sz = (int64_t)a.n[0] * a.n[1];
        const int g0 = ghost(q0, a.n[0], a.periodic[0]), g1 = ghost(q1, a.n[1], a.periodic[1]);
        const int64_t cxy = g0 + sy * g1;
        const int64_t oxm = ghost(q0 - 1, a.n[0], a.periodic[0]) - g0;
        const int64_t oxp = ghost(q0 + 1, a.n[0], a.periodic[0]) - g0;
        const int64_t oym = sy * (ghost(q1 - 1, a.n[1], a.periodic[1]) - g1);
        const int64_t oyp = sy * (ghost(q1 + 1, a.n[1], a.periodic[1]) - g1);
        auto plane = [&](int q2) -> int64_t { return cxy + sz * ghost(q2, a.n[2], a.periodic[2]); };
        T zm[4], z0s[4], zp[4];
        // extended plane ze holds coordinate q2 = ze - 1; its z stencil is q2-1 .. q2+1, all in [-2, n2+1]
        load4(a.u, plane(z0 - 2), zm);
        load4(a.u, plane(z0 - 1), z0s);
        for (int ze = z0; ze < z1; ze++) {
            const int64_t i0 = plane(ze - 1);
            T xm[4], xp[4], ym[4], yp[4];
            load4(a.u, plane(ze), zp);
            load4(a.u, i0 + oxm, xm);
            load4(a.u, i0 + oxp, xp);
            load4(a.u, i0 + oym, ym);
            load4(a.u, i0 + oyp, yp);
            T delta[4] = {T(0), T(0), T(0), T(0)};
            unsplit_axis<0, LIM>(a, eos, xm, z0s, xp, delta, cnt);
            unsplit_axis<1, LIM>(a, eos, ym, z0s, yp, delta, cnt);
            unsplit_axis<2, LIM>(a, eos, zm, z0s, zp, delta, cnt);
            const int64_t e = col + (int64_t)ze * ex * ey;
#pragma unroll
            for (int c = 0; c < 4; c++) a.dl[c * a.dl_n + e] = delta[c];
            copy4(z0s, zm);
            copy4(zp, z0s);
        }
    }
    flush_stats(a.stats, cnt, T(0), false);
}

// ---------------------------------------------------------------------------
// Batched sweeps: one persistent launch per axis sweep over every event of a
// handle.  The tiles of event e are [tile_start[e], tile_start[e+1]); a tile
// is one block's work of the per-event kernels (256 or 128 lines x one
// segment for y and z, block/64 wavefronts of row items for x).  Blocks pop
// tiles from an atomic counter until the queue is empty, so uneven events
// balance across the compute units; the arithmetic per cell is that of the
// per-event kernels.
// ---------------------------------------------------------------------------
template <typename T, int D, int LIM, class Eos, bool JET>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sweep_waves<Eos, JET>())))
void k_batch_sweep(const SweepArgs<T>* __restrict__ tab, const int64_t* __restrict__ tile_start, int ne,
                   unsigned int* counter, Eos eos)
{
    __shared__ int64_t sh_tile;
    __shared__ double eos_cache[Eos::kCacheDoubles];
    eos.bind_cache(eos_cache);
    const int64_t total = tile_start[ne];
    for (;;) {
        if (threadIdx.x == 0) sh_tile = (int64_t)atomicAdd(counter, 1u);
        __syncthreads();
        const int64_t tile = sh_tile;
        __syncthreads();
        if (tile >= total) break;
        int lo = 0, hi = ne;  // tile_start[lo] <= tile < tile_start[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (tile_start[mid] <= tile) lo = mid;
            else hi = mid;
        }
        const SweepArgs<T>& a = tab[lo];
        const int64_t local = tile - tile_start[lo];
        Counts cnt;
        T smax = T(0);
        if constexpr (D == 0) {
            __shared__ T carry[256 / 64][8];
            const int64_t wave = local * (blockDim.x >> 6) + (threadIdx.x >> 6);
            sweep_x_wave<T, LIM, Eos>(a, eos, wave, threadIdx.x & 63, carry[threadIdx.x >> 6], cnt, smax);
        } else {
            const int64_t nbx = (a.nlines + blockDim.x - 1) / blockDim.x;
            const int64_t bx = local % nbx, by = local / nbx;
            sweep_line<T, D, LIM, Eos, JET>(a, eos, bx * blockDim.x + threadIdx.x, (int)by * a.seg, cnt, smax);
        }
        flush_stats(a.stats, cnt, smax, sweep_mode<D>() == SW_FINAL && a.want_smax);
    }
}

__global__ void k_advance_time(double* t, const double* dt, int ne)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ne) t[i] = t[i] + dt[i];
}

__global__ void k_fill_u32(unsigned int* p, int n, unsigned int v)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// Standalone con2prim (Sec. 2.6) over n states.
// ---------------------------------------------------------------------------
// With the charge (NC = 5) the rest-frame density n = R sqrt(1 - v^2) goes to prim[5].
template <typename T, class Eos, int NC = 4>
__global__ __launch_bounds__(256) void k_con2prim(C2PArgs<T> a, Eos eos)
{
    __shared__ double eos_cache[Eos::kCacheDoubles];
    eos.bind_cache(eos_cache);
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    Counts cnt;
    if (i < a.n) {
        T u[NC];
        loadn<NC>(a.U, i, u);
        T e, p, v[3], cs2;
        Counts c1;
        eos.prim(u, e, p, v, cs2, c1);
        a.prim[0][i] = e; a.prim[1][i] = p;
        a.prim[2][i] = v[0]; a.prim[3][i] = v[1]; a.prim[4][i] = v[2];
        if constexpr (NC == 5) {
            // a non-finite charge makes the state bad; a zero state has n = 0 like its other primitives
            bool live = c1.bad == 0;
            if (live && !(fabs(u[4]) <= big_value<T>())) {
                c1.bad += 1;
                live = false;
                a.prim[0][i] = T(0); a.prim[1][i] = T(0);
                a.prim[2][i] = T(0); a.prim[3][i] = T(0); a.prim[4][i] = T(0);
            }
            a.prim[5][i] = live ? u[4] * Math<T>::sqrt(T(1) - (v[0] * v[0] + v[1] * v[1] + v[2] * v[2])) : T(0);
        }
        if (a.iters) a.iters[i] = (int32_t)c1.iters;
        add_counts(cnt, c1);
    }
    flush_stats(a.stats, cnt, T(0), false);
}

// ---------------------------------------------------------------------------
// Conservation sums: fixed assignment of cells to threads, fixed-order tree
// in LDS, one partial per block; the final kernel sums the partials in order.
// ---------------------------------------------------------------------------
template <typename T, int NC>
__global__ __launch_bounds__(256) void k_totals_partial(TotalsArgs<T> a)
{
    __shared__ double sh[NC][256];
    const int t = threadIdx.x;
    double s[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) s[c] = 0.0;
    const int64_t chunk = (a.n + gridDim.x - 1) / gridDim.x;
    const int64_t lo = (int64_t)blockIdx.x * chunk;
    const int64_t hi = min(lo + chunk, a.n);
    for (int64_t i = lo + t; i < hi; i += 256) {
#pragma unroll
        for (int c = 0; c < NC; c++) s[c] += (double)a.U[c][i];
    }
#pragma unroll
    for (int c = 0; c < NC; c++) sh[c][t] = s[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
#pragma unroll
            for (int c = 0; c < NC; c++) sh[c][t] += sh[c][t + w];
        }
        __syncthreads();
    }
    if (t < NC) a.partial[(int64_t)blockIdx.x * NC + t] = sh[t][0];
}

template <int NC>
__global__ __launch_bounds__(256) void k_totals_final(const double* partial, int nblocks, double dV,
                                                       double* out)
{
    __shared__ double sh[NC][256];
    const int t = threadIdx.x;
    double s[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) s[c] = 0.0;
    for (int b = t; b < nblocks; b += 256) {
#pragma unroll
        for (int c = 0; c < NC; c++) s[c] += partial[(int64_t)b * NC + c];
    }
#pragma unroll
    for (int c = 0; c < NC; c++) sh[c][t] = s[c];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
#pragma unroll
            for (int c = 0; c < NC; c++) sh[c][t] += sh[c][t + w];
        }
        __syncthreads();
    }
    if (t < NC) out[t] = sh[t][0] * dV;
}

__global__ void k_fill_u64(unsigned long long* p, int64_t n, unsigned long long v)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// Host-side launchers
// ---------------------------------------------------------------------------
template <typename T, int D, int LIM, class Eos>
static hipError_t launch_lim(bool jet, dim3 grid, dim3 block, hipStream_t s, const SweepArgs<T>& a,
                             const Eos& eos)
{
    if constexpr (D == 0) {
        hipLaunchKernelGGL((k_sweep_x<T, LIM, Eos>), grid, block, 0, s, a, eos);
    } else if constexpr (D == 2) {
        if (jet) hipLaunchKernelGGL((k_sweep<T, D, LIM, Eos, true>), grid, block, 0, s, a, eos);
        else hipLaunchKernelGGL((k_sweep<T, D, LIM, Eos, false>), grid, block, 0, s, a, eos);
    } else {
        hipLaunchKernelGGL((k_sweep<T, D, LIM, Eos, false>), grid, block, 0, s, a, eos);
    }
    return hipGetLastError();
}

template <typename T, int D, class Eos>
static hipError_t launch_axis(int lim, bool jet, dim3 grid, dim3 block, hipStream_t s,
                              const SweepArgs<T>& a, const Eos& eos)
{
    switch (lim) {
    case LIM_NONE: return launch_lim<T, D, LIM_NONE>(jet, grid, block, s, a, eos);
    case LIM_MINMOD: return launch_lim<T, D, LIM_MINMOD>(jet, grid, block, s, a, eos);
    case LIM_SUPERBEE: return launch_lim<T, D, LIM_SUPERBEE>(jet, grid, block, s, a, eos);
    case LIM_MC: return launch_lim<T, D, LIM_MC>(jet, grid, block, s, a, eos);
    case LIM_VANLEER: return launch_lim<T, D, LIM_VANLEER>(jet, grid, block, s, a, eos);
    case LIM_VANALBADA: return launch_lim<T, D, LIM_VANALBADA>(jet, grid, block, s, a, eos);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, class Eos>
hipError_t launch_sweep(int axis, int lim, bool jet, dim3 grid, dim3 block, hipStream_t s,
                        const SweepArgs<T>& a, const Eos& eos)
{
    switch (axis) {
    case 0: return launch_axis<T, 0>(lim, false, grid, block, s, a, eos);
    case 1: return launch_axis<T, 1>(lim, false, grid, block, s, a, eos);
    case 2: return launch_axis<T, 2>(lim, jet, grid, block, s, a, eos);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int LIM, class Eos>
static int x_waves_lim(int block)
{
    static int w[3] = {0, 0, 0};  // by block size 64 / 128 / 256
    const int bi = block == 64 ? 0 : (block == 128 ? 1 : 2);
    if (w[bi] == 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(&k_sweep_x<T, LIM, Eos>),
                                                         block, 0) != hipSuccess || nb < 1)
            nb = 1;
        w[bi] = std::max(1, nb * (block / 64) / 4);
    }
    return w[bi];
}

template <typename T, class Eos>
int sweep_x_waves(int lim, int block);

template <typename T, int D, int LIM, class Eos, bool JET>
static int yz_waves_lim(int block)
{
    static int w[3] = {0, 0, 0};  // by block size 64 / 128 / 256
    const int bi = block == 64 ? 0 : (block == 128 ? 1 : 2);
    if (w[bi] == 0) {
        int nb = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &nb, reinterpret_cast<const void*>(&k_sweep<T, D, LIM, Eos, JET>), block, 0) != hipSuccess || nb < 1)
            nb = 1;
        w[bi] = std::max(1, nb * (block / 64) / 4);
    }
    return w[bi];
}

template <typename T, int D, class Eos, bool JET>
static int yz_waves_axis(int lim, int block)
{
    switch (lim) {
    case LIM_NONE: return yz_waves_lim<T, D, LIM_NONE, Eos, JET>(block);
    case LIM_MINMOD: return yz_waves_lim<T, D, LIM_MINMOD, Eos, JET>(block);
    case LIM_SUPERBEE: return yz_waves_lim<T, D, LIM_SUPERBEE, Eos, JET>(block);
    case LIM_MC: return yz_waves_lim<T, D, LIM_MC, Eos, JET>(block);
    case LIM_VANLEER: return yz_waves_lim<T, D, LIM_VANLEER, Eos, JET>(block);
    default: return yz_waves_lim<T, D, LIM_VANALBADA, Eos, JET>(block);
    }
}

template <typename T, class Eos>
int sweep_waves_per_simd(int axis, int lim, bool jet, int block)
{
    if (axis == 1) return yz_waves_axis<T, 1, Eos, false>(lim, block);
    if (axis == 2) return jet ? yz_waves_axis<T, 2, Eos, true>(lim, block) : yz_waves_axis<T, 2, Eos, false>(lim, block);
    return sweep_x_waves<T, Eos>(lim, block);
}

template <typename T, class Eos>
int sweep_x_waves(int lim, int block)
{
    switch (lim) {
    case LIM_NONE: return x_waves_lim<T, LIM_NONE, Eos>(block);
    case LIM_MINMOD: return x_waves_lim<T, LIM_MINMOD, Eos>(block);
    case LIM_SUPERBEE: return x_waves_lim<T, LIM_SUPERBEE, Eos>(block);
    case LIM_MC: return x_waves_lim<T, LIM_MC, Eos>(block);
    case LIM_VANLEER: return x_waves_lim<T, LIM_VANLEER, Eos>(block);
    default: return x_waves_lim<T, LIM_VANALBADA, Eos>(block);
    }
}

template <typename T, int LIM, class Eos>
static hipError_t launch_unsplit_lim(bool jet, int axis, dim3 grid, dim3 block, hipStream_t s, const SweepArgs<T>& a,
                                     const Eos& eos)
{
    if (axis == 0) hipLaunchKernelGGL((k_sweep_x<T, LIM, Eos, true>), grid, block, 0, s, a, eos);
    else if (axis == 1) hipLaunchKernelGGL((k_sweep<T, 1, LIM, Eos, false, true>), grid, block, 0, s, a, eos);
    else if (jet) hipLaunchKernelGGL((k_sweep<T, 2, LIM, Eos, true, true>), grid, block, 0, s, a, eos);
    else hipLaunchKernelGGL((k_sweep<T, 2, LIM, Eos, false, true>), grid, block, 0, s, a, eos);
    return hipGetLastError();
}

template <typename T, class Eos>
hipError_t launch_sweep_unsplit(int axis, int lim, bool jet, dim3 grid, dim3 block, hipStream_t s,
                                const SweepArgs<T>& a, const Eos& eos)
{
    if (axis < 0 || axis > 2) return hipErrorInvalidValue;
    switch (lim) {
    case LIM_NONE: return launch_unsplit_lim<T, LIM_NONE>(jet, axis, grid, block, s, a, eos);
    case LIM_MINMOD: return launch_unsplit_lim<T, LIM_MINMOD>(jet, axis, grid, block, s, a, eos);
    case LIM_SUPERBEE: return launch_unsplit_lim<T, LIM_SUPERBEE>(jet, axis, grid, block, s, a, eos);
    case LIM_MC: return launch_unsplit_lim<T, LIM_MC>(jet, axis, grid, block, s, a, eos);
    case LIM_VANLEER: return launch_unsplit_lim<T, LIM_VANLEER>(jet, axis, grid, block, s, a, eos);
    case LIM_VANALBADA: return launch_unsplit_lim<T, LIM_VANALBADA>(jet, axis, grid, block, s, a, eos);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, class Eos>
hipError_t launch_unsplit_delta(int lim, hipStream_t s, const UnsplitArgs<T>& a0, const Eos& eos)
{
    constexpr int kZSeg = 8;
    UnsplitArgs<T> a = a0;
    a.zseg = kZSeg;
    const int64_t cols = (int64_t)(a.n[0] + 2) * (a.n[1] + 2);
    const int64_t chunks = (cols + 255) / 256;
    const dim3 grid((unsigned)(8 * ((chunks + 7) / 8)), (unsigned)((a.n[2] + 2 + kZSeg - 1) / kZSeg)), block(256);
    switch (lim) {
    case LIM_NONE: hipLaunchKernelGGL((k_unsplit_delta<T, LIM_NONE, Eos>), grid, block, 0, s, a, eos); break;
    case LIM_MINMOD: hipLaunchKernelGGL((k_unsplit_delta<T, LIM_MINMOD, Eos>), grid, block, 0, s, a, eos); break;
    case LIM_SUPERBEE: hipLaunchKernelGGL((k_unsplit_delta<T, LIM_SUPERBEE, Eos>), grid, block, 0, s, a, eos); break;
    case LIM_MC: hipLaunchKernelGGL((k_unsplit_delta<T, LIM_MC, Eos>), grid, block, 0, s, a, eos); break;
    case LIM_VANLEER: hipLaunchKernelGGL((k_unsplit_delta<T, LIM_VANLEER, Eos>), grid, block, 0, s, a, eos); break;
    case LIM_VANALBADA: hipLaunchKernelGGL((k_unsplit_delta<T, LIM_VANALBADA, Eos>), grid, block, 0, s, a, eos); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <typename T, class Eos>
hipError_t launch_con2prim(int64_t n, hipStream_t s, const C2PArgs<T>& a, const Eos& eos)
{
    const int64_t nb = (n + 255) / 256;
    hipLaunchKernelGGL((k_con2prim<T, Eos>), dim3((unsigned)nb), dim3(256), 0, s, a, eos);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_totals(hipStream_t s, const TotalsArgs<T>& a, int nc, int nblocks, double dV, double* out)
{
    if (nc == 5) hipLaunchKernelGGL((k_totals_partial<T, 5>), dim3(nblocks), dim3(256), 0, s, a);
    else hipLaunchKernelGGL((k_totals_partial<T, 4>), dim3(nblocks), dim3(256), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (nc == 5) hipLaunchKernelGGL(k_totals_final<5>, dim3(1), dim3(256), 0, s, a.partial, nblocks, dV, out);
    else hipLaunchKernelGGL(k_totals_final<4>, dim3(1), dim3(256), 0, s, a.partial, nblocks, dV, out);
    return hipGetLastError();
}

hipError_t launch_fill_u64(hipStream_t s, unsigned long long* p, int64_t n, unsigned long long v)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}


template <typename T, int D, int LIM, class Eos, bool JET>
static hipError_t launch_batch_lim(const SweepArgs<T>* tab, const int64_t* tile_start, int ne, unsigned int* counter,
                                   int64_t total_tiles, int block, hipStream_t s, const Eos& eos)
{
    static int per_cu[3] = {0, 0, 0};  // resident blocks per CU, by block size 64/128/256
    static int n_cu = 0;
    const int bi = block == 64 ? 0 : (block == 128 ? 1 : 2);
    if (per_cu[bi] == 0) {
        int nb = 0;
        hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(
            &nb, reinterpret_cast<const void*>(&k_batch_sweep<T, D, LIM, Eos, JET>), block, 0);
        if (e != hipSuccess) return e;
        per_cu[bi] = nb > 0 ? nb : 1;
        if (n_cu == 0) {
            int dev = 0;
            (void)hipGetDevice(&dev);
            e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
            if (e != hipSuccess) return e;
        }
    }
    const int64_t grid = std::min<int64_t>(total_tiles, (int64_t)per_cu[bi] * n_cu);
    if (grid <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_batch_sweep<T, D, LIM, Eos, JET>), dim3((unsigned)grid), dim3(block), 0, s, tab, tile_start,
                       ne, counter, eos);
    return hipGetLastError();
}

template <typename T, int D, class Eos>
static hipError_t launch_batch_axis(int lim, bool jet, const SweepArgs<T>* tab, const int64_t* tile_start, int ne,
                                    unsigned int* counter, int64_t total_tiles, int block, hipStream_t s,
                                    const Eos& eos)
{
#define MF_BATCH_CASE(L)                                                                                      \
    case L:                                                                                                  \
        if constexpr (D == 2) {                                                                              \
            if (jet) return launch_batch_lim<T, D, L, Eos, true>(tab, tile_start, ne, counter, total_tiles,    \
                                                                 block, s, eos);                              \
        }                                                                                                    \
        return launch_batch_lim<T, D, L, Eos, false>(tab, tile_start, ne, counter, total_tiles, block, s, eos);
    switch (lim) {
        MF_BATCH_CASE(LIM_NONE)
        MF_BATCH_CASE(LIM_MINMOD)
        MF_BATCH_CASE(LIM_SUPERBEE)
        MF_BATCH_CASE(LIM_MC)
        MF_BATCH_CASE(LIM_VANLEER)
        MF_BATCH_CASE(LIM_VANALBADA)
    default: return hipErrorInvalidValue;
    }
#undef MF_BATCH_CASE
}

template <typename T, class Eos>
hipError_t launch_batch_sweep(int axis, int lim, bool jet, const SweepArgs<T>* tab, const int64_t* tile_start, int ne,
                              unsigned int* counter, int64_t total_tiles, int block, hipStream_t s, const Eos& eos)
{
    switch (axis) {
    case 0: return launch_batch_axis<T, 0>(lim, false, tab, tile_start, ne, counter, total_tiles, block, s, eos);
    case 1: return launch_batch_axis<T, 1>(lim, false, tab, tile_start, ne, counter, total_tiles, block, s, eos);
    case 2: return launch_batch_axis<T, 2>(lim, jet, tab, tile_start, ne, counter, total_tiles, block, s, eos);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_advance_time(hipStream_t s, double* t, const double* dt, int ne)
{
    hipLaunchKernelGGL(k_advance_time, dim3((ne + 63) / 64), dim3(64), 0, s, t, dt, ne);
    return hipGetLastError();
}

hipError_t launch_fill_u32(hipStream_t s, unsigned int* p, int n, unsigned int v)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u32, dim3((n + 63) / 64), dim3(64), 0, s, p, n, v);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Sweeps with the conserved charge (5 components; FP64, per event, no jet):
// p = e/3 with a passive charge (EosIdeal<double>) or the ideal gas (EosGamma).
// ---------------------------------------------------------------------------
template <int D, int LIM, class Eos>
static hipError_t launch_charge_lim(dim3 grid, dim3 block, hipStream_t s, const SweepArgs<double>& a, const Eos& eos)
{
    if constexpr (D == 0) hipLaunchKernelGGL((k_sweep_x<double, LIM, Eos, false, 5>), grid, block, 0, s, a, eos);
    else hipLaunchKernelGGL((k_sweep<double, D, LIM, Eos, false, false, 5>), grid, block, 0, s, a, eos);
    return hipGetLastError();
}

template <int D, int LIM, class Eos>
static int charge_waves_lim(int block)
{
    static int w[3] = {0, 0, 0};  // by block size 64 / 128 / 256
    const int bi = block == 64 ? 0 : (block == 128 ? 1 : 2);
    if (w[bi] == 0) {
        int nb = 0;
        const void* k = D == 0 ? reinterpret_cast<const void*>(&k_sweep_x<double, LIM, Eos, false, 5>)
                               : reinterpret_cast<const void*>(&k_sweep<double, D, LIM, Eos, false, false, 5>);
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, block, 0) != hipSuccess || nb < 1) nb = 1;
        w[bi] = std::max(1, nb * (block / 64) / 4);
    }
    return w[bi];
}

template <int LIM, class Eos>
static hipError_t launch_charge_axis(int axis, dim3 grid, dim3 block, hipStream_t s, const SweepArgs<double>& a,
                                     const Eos& eos)
{
    switch (axis) {
    case 0: return launch_charge_lim<0, LIM>(grid, block, s, a, eos);
    case 1: return launch_charge_lim<1, LIM>(grid, block, s, a, eos);
    case 2: return launch_charge_lim<2, LIM>(grid, block, s, a, eos);
    default: return hipErrorInvalidValue;
    }
}

template <int LIM, class Eos>
static int charge_waves_axis(int axis, int block)
{
    switch (axis) {
    case 0: return charge_waves_lim<0, LIM, Eos>(block);
    case 1: return charge_waves_lim<1, LIM, Eos>(block);
    default: return charge_waves_lim<2, LIM, Eos>(block);
    }
}

template <class Eos>
hipError_t launch_sweep_charge(int axis, int lim, dim3 grid, dim3 block, hipStream_t s, const SweepArgs<double>& a,
                               const Eos& eos)
{
    switch (lim) {
    case LIM_NONE: return launch_charge_axis<LIM_NONE>(axis, grid, block, s, a, eos);
    case LIM_MINMOD: return launch_charge_axis<LIM_MINMOD>(axis, grid, block, s, a, eos);
    case LIM_SUPERBEE: return launch_charge_axis<LIM_SUPERBEE>(axis, grid, block, s, a, eos);
    case LIM_MC: return launch_charge_axis<LIM_MC>(axis, grid, block, s, a, eos);
    case LIM_VANLEER: return launch_charge_axis<LIM_VANLEER>(axis, grid, block, s, a, eos);
    case LIM_VANALBADA: return launch_charge_axis<LIM_VANALBADA>(axis, grid, block, s, a, eos);
    default: return hipErrorInvalidValue;
    }
}

template <class Eos>
int sweep_waves_per_simd_charge(int axis, int lim, int block)
{
    switch (lim) {
    case LIM_NONE: return charge_waves_axis<LIM_NONE, Eos>(axis, block);
    case LIM_MINMOD: return charge_waves_axis<LIM_MINMOD, Eos>(axis, block);
    case LIM_SUPERBEE: return charge_waves_axis<LIM_SUPERBEE, Eos>(axis, block);
    case LIM_MC: return charge_waves_axis<LIM_MC, Eos>(axis, block);
    case LIM_VANLEER: return charge_waves_axis<LIM_VANLEER, Eos>(axis, block);
    default: return charge_waves_axis<LIM_VANALBADA, Eos>(axis, block);
    }
}

template <class Eos>
hipError_t launch_con2prim_charge(int64_t n, hipStream_t s, const C2PArgs<double>& a, const Eos& eos)
{
    const int64_t nb = (n + 255) / 256;
    hipLaunchKernelGGL((k_con2prim<double, Eos, 5>), dim3((unsigned)nb), dim3(256), 0, s, a, eos);
    return hipGetLastError();
}

template hipError_t launch_sweep_charge<EosIdeal<double>>(int, int, dim3, dim3, hipStream_t, const SweepArgs<double>&,
                                                          const EosIdeal<double>&);
template hipError_t launch_sweep_charge<EosGamma>(int, int, dim3, dim3, hipStream_t, const SweepArgs<double>&,
                                                  const EosGamma&);
template int sweep_waves_per_simd_charge<EosIdeal<double>>(int, int, int);
template int sweep_waves_per_simd_charge<EosGamma>(int, int, int);
template hipError_t launch_con2prim_charge<EosIdeal<double>>(int64_t, hipStream_t, const C2PArgs<double>&,
                                                             const EosIdeal<double>&);
template hipError_t launch_con2prim_charge<EosGamma>(int64_t, hipStream_t, const C2PArgs<double>&, const EosGamma&);

template hipError_t launch_batch_sweep<double, EosIdeal<double>>(int, int, bool, const SweepArgs<double>*,
                                                                 const int64_t*, int, unsigned int*, int64_t, int,
                                                                 hipStream_t, const EosIdeal<double>&);
template hipError_t launch_batch_sweep<float, EosIdeal<float>>(int, int, bool, const SweepArgs<float>*, const int64_t*,
                                                               int, unsigned int*, int64_t, int, hipStream_t,
                                                               const EosIdeal<float>&);
template hipError_t launch_batch_sweep<double, EosTable>(int, int, bool, const SweepArgs<double>*, const int64_t*,
                                                         int, unsigned int*, int64_t, int, hipStream_t,
                                                         const EosTable&);

template hipError_t launch_sweep<double, EosIdeal<double>>(int, int, bool, dim3, dim3, hipStream_t,
                                                           const SweepArgs<double>&, const EosIdeal<double>&);
template hipError_t launch_sweep<float, EosIdeal<float>>(int, int, bool, dim3, dim3, hipStream_t,
                                                         const SweepArgs<float>&, const EosIdeal<float>&);
template hipError_t launch_sweep<double, EosTable>(int, int, bool, dim3, dim3, hipStream_t,
                                                   const SweepArgs<double>&, const EosTable&);
template int sweep_waves_per_simd<double, EosIdeal<double>>(int, int, bool, int);
template int sweep_waves_per_simd<float, EosIdeal<float>>(int, int, bool, int);
template int sweep_waves_per_simd<double, EosTable>(int, int, bool, int);
template hipError_t launch_sweep_unsplit<double, EosIdeal<double>>(int, int, bool, dim3, dim3, hipStream_t,
                                                                   const SweepArgs<double>&, const EosIdeal<double>&);
template hipError_t launch_sweep_unsplit<float, EosIdeal<float>>(int, int, bool, dim3, dim3, hipStream_t,
                                                                 const SweepArgs<float>&, const EosIdeal<float>&);
template hipError_t launch_sweep_unsplit<double, EosTable>(int, int, bool, dim3, dim3, hipStream_t,
                                                           const SweepArgs<double>&, const EosTable&);
template hipError_t launch_unsplit_delta<double, EosIdeal<double>>(int, hipStream_t, const UnsplitArgs<double>&,
                                                                   const EosIdeal<double>&);
template hipError_t launch_unsplit_delta<float, EosIdeal<float>>(int, hipStream_t, const UnsplitArgs<float>&,
                                                                 const EosIdeal<float>&);
template hipError_t launch_unsplit_delta<double, EosTable>(int, hipStream_t, const UnsplitArgs<double>&,
                                                           const EosTable&);
template hipError_t launch_con2prim<double, EosIdeal<double>>(int64_t, hipStream_t, const C2PArgs<double>&,
                                                              const EosIdeal<double>&);
template hipError_t launch_con2prim<float, EosIdeal<float>>(int64_t, hipStream_t, const C2PArgs<float>&,
                                                            const EosIdeal<float>&);
template hipError_t launch_con2prim<double, EosTable>(int64_t, hipStream_t, const C2PArgs<double>&,
                                                      const EosTable&);
template hipError_t launch_totals<double>(hipStream_t, const TotalsArgs<double>&, int, int, double, double*);
template hipError_t launch_totals<float>(hipStream_t, const TotalsArgs<float>&, int, int, double, double*);

}  // namespace mf
