// mf_device.hpp -- pointwise device building blocks of the MUSTA-FORCE step
// for gfx950: conserved-to-primitive recovery, physical fluxes, slope
// limiters, the Hancock half step and the MUSTA-FORCE interface flux.
//
// Everything here is register-resident and templated on the arithmetic type
// T (double or float) and on the sweep axis D (0 = x, 1 = y, 2 = z).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mf_params.hpp"

namespace mf {

enum { LIM_NONE = 0, LIM_MINMOD, LIM_SUPERBEE, LIM_MC, LIM_VANLEER, LIM_VANALBADA };

// ---------------------------------------------------------------------------
// Reciprocal and square root.  FP64: the hardware estimates (v_rcp_f64,
// v_rsq_f64) refined by Newton-Raphson steps in FMA, which is within an ulp of
// the IEEE results for the normal, positive arguments met here (denominators
// >= E > 0), without the scaling and fix-up code of the IEEE expansions.
// FP32: the hardware instructions (about 1 ulp).
// ---------------------------------------------------------------------------
template <typename T> struct Math;

template <> struct Math<double> {
    static __device__ __forceinline__ double rcp(double x)
    {
        double r = __builtin_amdgcn_rcp(x);
        double e = __builtin_fma(-x, r, 1.0);
        r = __builtin_fma(r, e, r);
        e = __builtin_fma(-x, r, 1.0);
        return __builtin_fma(r, e, r);
    }
    static __device__ __forceinline__ double sqrt(double x)
    {
        double y = __builtin_amdgcn_rsq(x);
        double g = x * y;          // sqrt(x) estimate
        double h = 0.5 * y;        // 1 / (2 sqrt(x)) estimate
        double r = __builtin_fma(-g, h, 0.5);
        g = __builtin_fma(g, r, g);
        h = __builtin_fma(h, r, h);
        double d = __builtin_fma(-g, g, x);
        return __builtin_fma(d, h, g);
    }
    // sqrt(x) as sqrt() gives it, and 1/sqrt(x) from the same Goldschmidt step
    // (2h, relative error about 1e-15: for derivatives, not for results).
    static __device__ __forceinline__ double sqrt_rsq(double x, double& rs)
    {
        double y = __builtin_amdgcn_rsq(x);
        double g = x * y;
        double h = 0.5 * y;
        double r = __builtin_fma(-g, h, 0.5);
        g = __builtin_fma(g, r, g);
        h = __builtin_fma(h, r, h);
        double d = __builtin_fma(-g, g, x);
        rs = 2.0 * h;
        return __builtin_fma(d, h, g);
    }
    // sqrt that also returns 0 for x == 0 (rsq(0) is +inf).
    static __device__ __forceinline__ double sqrt0(double x) { return x > 0.0 ? sqrt(x) : 0.0; }
    // sqrt for any x >= 0: below 2^-767 (where the hardware estimate does not hold, e.g. the
    // squared momenta of near-vacuum states) the argument is scaled by 2^256 and the result
    // by 2^-128, which is exact.  For the guards' slow paths, not the common path.
    static __device__ __forceinline__ double sqrt_safe(double x)
    {
        const bool tiny = x < 0x1p-767;
        const double r = sqrt0(tiny ? x * 0x1p+256 : x);
        return tiny ? r * 0x1p-128 : r;
    }
    static __device__ __forceinline__ double div(double a, double b) { return a / b; }
};

template <> struct Math<float> {
    static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
    static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float sqrt0(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float sqrt_safe(float x) { return __builtin_amdgcn_sqrtf(x); }
    static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
};

// Wavefront votes.  The ballot of one compare stays a lane mask in scalar
// registers; the ballot of a combined condition (a & b) is first copied
// through a vector register (two more vector instructions), so a guard made
// of several compares takes one ballot per compare and ORs the masks.
__device__ __forceinline__ uint64_t lanes_where(bool c) { return __builtin_amdgcn_ballot_w64(c); }
__device__ __forceinline__ bool lane_in(uint64_t mask)
{
    const unsigned lane = __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u));
    return (mask >> lane) & 1u;
}

template <typename T> __device__ __forceinline__ T big_value();
template <> __device__ __forceinline__ double big_value<double>() { return 1.79769313486231570e308; }
template <> __device__ __forceinline__ float big_value<float>() { return 3.40282347e38f; }

// Near-vacuum states: below tiny_value the square E^2 (and |M|^2) leaves the
// range where the hardware reciprocal and square-root estimates hold, so such
// states are evaluated scaled up by an exact power of two (up_scale) and their
// fluxes and energies scaled back (down_scale).  con2prim of p = c e and of the
// ideal gas is invariant under that scaling (v is unchanged, e, n, p and the
// fluxes scale with the state); a table EoS is linear there (far below its
// first node).  Chosen so that every positive double below tiny_value lands,
// with its square, in the normal range above 2^-767.
template <typename T> __device__ __forceinline__ T tiny_value();
template <> __device__ __forceinline__ double tiny_value<double>() { return 0x1p-380; }
template <> __device__ __forceinline__ float tiny_value<float>() { return 0x1p-60f; }
template <typename T> __device__ __forceinline__ T up_scale();
template <> __device__ __forceinline__ double up_scale<double>() { return 0x1p+700; }
template <> __device__ __forceinline__ float up_scale<float>() { return 0x1p+100f; }
template <typename T> __device__ __forceinline__ T down_scale();
template <> __device__ __forceinline__ double down_scale<double>() { return 0x1p-700; }
template <> __device__ __forceinline__ float down_scale<float>() { return 0x1p-100f; }

// Largest admitted |M| / E; larger momenta are scaled down to it for the
// evaluation (the stored state is not changed).
template <typename T> __device__ __forceinline__ T mmax();
template <> __device__ __forceinline__ double mmax<double>() { return 1.0 - 1e-12; }
template <> __device__ __forceinline__ float mmax<float>() { return 1.0f - 1e-6f; }

// Per-thread counters of guarded states, kept in registers.
struct Counts {
    uint32_t floor_ = 0;  // |M| clamped
    uint32_t bad = 0;     // E <= 0 or non-finite
    uint32_t iters = 0;   // root-finder iterations (table EoS)
    uint32_t fallback = 0; // seeded solves whose guess lay outside the bracket
    uint32_t w = 1;       // added per event: 0 where the evaluation is not counted
                          // (segment overlaps of the sweeps)
};

// ---------------------------------------------------------------------------
// Equations of state.  An EoS provides
//   flux<D, NC>(U, F, counts):  F = F_D(U) after con2prim, for NC = 4
//       components (E, Mx, My, Mz) or 5 (with the charge R, flux R v_D);
//   prim(U, e, p, v[3], cs2, counts): full primitive recovery.
// ---------------------------------------------------------------------------

// p = c e.  con2prim of the fixed point v = |M| / (E + p(E - |M| v)) is the
// root below one of  c|M| v^2 - (1+c) E v + |M| = 0:
//   v_vec = 2 M / ((1+c) E + sqrt((1+c)^2 E^2 - 4 c |M|^2)),  e = E - M.v.
template <typename T> struct EosIdeal {
    static constexpr int kWaves = 4;  // sweep kernels fit 128 VGPRs without spilling
    static constexpr bool kLoadLAhead = false;  // no gain at 4 waves; FP32 would lose a wave
    static constexpr int kCacheDoubles = 1;  // no lookup cache
    __device__ __forceinline__ void bind_cache(double*) const {}
    T c;    // cs2
    T qh;   // (1 + cs2) / 2
    T q2q;  // (1 + cs2)^2 / 4

    static EosIdeal make(double cs2)
    {
        EosIdeal e;
        e.c = (T)cs2;
        e.qh = (T)(0.5 * (1.0 + cs2));
        e.q2q = (T)(0.25 * (1.0 + cs2) * (1.0 + cs2));
        return e;
    }

    // With the halved radicand d = ((1+c)/2)^2 E^2 - c |M|^2 (= D/4, exact
    // scaling) the velocity is v_vec = M / ((1+c)/2 E + sqrt(d)).
    __device__ __forceinline__ T inv_half_den(T E, T E2, T M2) const
    {
        const T sd = Math<T>::sqrt(q2q * E2 - c * M2);
        return Math<T>::rcp(qh * E + sd);   // = 2 / ((1+c)E + sqrt(D))
    }

    // Guards (outside the common path): E <= 0 or non-finite input is counted
    // and evaluated as the zero state (zero flux, e = p = v = 0); |M| above
    // (1 - 1e-12) E is scaled down to that bound for this evaluation.
    // Returns false for the zero state.
    __device__ __forceinline__ bool fixup(T& E, T& Mx, T& My, T& Mz, T& M2, Counts& cnt) const
    {
        if (!((E > T(0)) & (E <= big_value<T>()) & (M2 <= big_value<T>()))) {
            cnt.bad += cnt.w;
            return false;
        }
        const T Mlim = mmax<T>() * E;
        if (M2 > Mlim * Mlim) {
            const T s = Math<T>::div(Mlim, Math<T>::sqrt_safe(M2));
            Mx = Mx * s; My = My * s; Mz = Mz * s;
            M2 = Mx * Mx + My * My + Mz * Mz;
            cnt.floor_ += cnt.w;
        }
        return true;
    }

    // The energy flux (E + p) v_D is M_D: r = 1 / (E + p) at the root.  Returns v_D.
    template <int D>
    __device__ __forceinline__ T flux_core(T E, T Mx, T My, T Mz, T M2, T F[4]) const
    {
        const T r = inv_half_den(E, E * E, M2);   // v_vec = r M
        const T e = E - r * M2;                   // E - M.v
        const T p = c * e;
        const T MD = (D == 0) ? Mx : ((D == 1) ? My : Mz);
        const T vD = r * MD;
        F[0] = MD;
        F[1] = Mx * vD;
        F[2] = My * vD;
        F[3] = Mz * vD;
        F[1 + D] = F[1 + D] + p;
        return vD;
    }

    // F = F_D(U) after con2prim.  The common path has no guard branches; when
    // any lane of the wavefront holds a state that needs a guard, those lanes
    // are re-evaluated on the slow path.  With the charge (NC = 5) p does not
    // depend on n, and the charge flux is R v_D.
    template <int D, int NC = 4>
    __device__ __forceinline__ void flux(const T u[], T F[], Counts& cnt) const
    {
        const T E = u[0], Mx = u[1], My = u[2], Mz = u[3];
        const T M2 = Mx * Mx + My * My + Mz * Mz;
        const T Mlim = mmax<T>() * E;
        // the first compare also sends near-vacuum states (E below tiny_value) to the slow path
        uint64_t bad = lanes_where(!(E >= tiny_value<T>())) | lanes_where(!(E <= big_value<T>())) |
                       lanes_where(!(M2 <= Mlim * Mlim));
        if constexpr (NC == 5) bad |= lanes_where(!(fabs(u[4]) <= big_value<T>()));
        const T vD = flux_core<D>(E, Mx, My, Mz, M2, F);
        if constexpr (NC == 5) F[4] = u[4] * vD;
        if (bad != 0) {
            if (lane_in(bad)) {
                const bool small = (E > T(0)) & (E < tiny_value<T>());
                const T sc = small ? up_scale<T>() : T(1);
                T Ef = E * sc, mx = Mx * sc, my = My * sc, mz = Mz * sc;
                T m2 = mx * mx + my * my + mz * mz;
                bool live = fixup(Ef, mx, my, mz, m2, cnt);
                if constexpr (NC == 5) {
                    if (live && !(fabs(u[4]) <= big_value<T>())) {
                        cnt.bad += cnt.w;
                        live = false;
                    }
                }
                if (live) {
                    const T vf = flux_core<D>(Ef, mx, my, mz, m2, F);
                    if (small) {
#pragma unroll
                        for (int c = 0; c < 4; c++) F[c] = F[c] * down_scale<T>();
                    }
                    if constexpr (NC == 5) F[4] = u[4] * vf;
                } else {
#pragma unroll
                    for (int c = 0; c < NC; c++) F[c] = T(0);
                }
            }
        }
    }

    // Fluxes of two independent states (CHAIN: see EosGamma::flux2).
    template <int D, int NC = 4, bool CHAIN = false>
    __device__ __forceinline__ void flux2(const T uA[], const T uB[], T FA[], T FB[], Counts& cnt) const
    {
        flux<D, NC>(uA, FA, cnt);
        flux<D, NC>(uB, FB, cnt);
    }
    // Flux of a state formed from the last pair (the closed form needs no start).
    template <int D, int NC = 4>
    __device__ __forceinline__ void flux_near(const T u[], T F[], Counts& cnt) const
    {
        flux<D, NC>(u, F, cnt);
    }

    __device__ __forceinline__ void prim(const T u[], T& e, T& p, T v[3], T& cs2, Counts& cnt) const
    {
        const bool small = (u[0] > T(0)) & (u[0] < tiny_value<T>());
        const T sc = small ? up_scale<T>() : T(1);
        T E = u[0] * sc, Mx = u[1] * sc, My = u[2] * sc, Mz = u[3] * sc;
        T M2 = Mx * Mx + My * My + Mz * Mz;
        cs2 = c;
        if (!fixup(E, Mx, My, Mz, M2, cnt)) {
            e = T(0); p = T(0); v[0] = T(0); v[1] = T(0); v[2] = T(0);
            return;
        }
        const T r = inv_half_den(E, E * E, M2);
        v[0] = r * Mx; v[1] = r * My; v[2] = r * Mz;
        e = E - (Mx * v[0] + My * v[1] + Mz * v[2]);
        if (small) e = e * down_scale<T>();
        p = c * e;
    }
};


// ---------------------------------------------------------------------------
// Tabulated p(e): monotone piecewise-cubic Hermite interpolation on nodes
// e_i with node slopes m_i (Fritsch-Carlson), p = p_0 e / e_0 below the first
// node and linear with the end slope above the last.
//
// The table holds n + 1 pieces of 48 bytes, (x, w), (y, c1), (c2, c3), with
// p(e) = y + t (c1 + t (c2 + t c3)), t = (e - x) w on [x, x + 1/w), i.e.
// 0 <= t < 1: piece 0 is the extrapolation below e_0 (x = 0, w = 1/e_0),
// pieces 1 .. n-1 the cubics between nodes (the Hermite cubic in powers of
// t), piece n the extrapolation above e_{n-1} (w = 2^-60, so t < 1 up to
// e ~ 1e18).  One piece is one lookup: three 16-byte loads.  A first-guess
// piece is accepted where 0 <= t < 1; elsewhere the piece is found by
// comparing e with the pieces' origins (exact), so either way e lies in the
// piece up to the rounding of t at its upper end, where the two cubics
// meeting at the node agree to rounding (the interpolant is C^1).
//
// con2prim (Sec. 2.6): the fixed point v = |M| / (E + p(E - |M| v)) is the
// root of g(e) = e - E + |M|^2 / (E + p(e)) on the bracket [E (1 - m^2), E],
// m = |M| / E (g is increasing there for dp/de < 1).  Safeguarded Newton from
// the bracket midpoint: stop when the Newton correction |de| <= 1e-7 e (the
// accepted iterate is then accurate to about 1e-14, see kNewtonTol) or
// |de| <= 1e-15 E (the rounding level of g);
// otherwise the bracket shrinks with the sign of g and a step that leaves it
// is replaced by bisection.  FP64 only.
// ---------------------------------------------------------------------------
struct EosTable {
    static constexpr int kWaves = 3;  // minimum waves per SIMD the sweeps are compiled for
    static constexpr bool kLoadLAhead = true;  // the y sweep loads L ahead (latency-bound at 3 waves)
    const double2* rec;  // 3 (n + 1) records: piece k = rec[3k] (x, w), rec[3k + 1] (y, c1), rec[3k + 2] (c2, c3)
    int32_t n;           // nodes
    int32_t log_uniform; // piece from log2(e) (then a fix-up); else bisection
    float lg0;           // log2 e_0 - (log2 e_{n-1} - log2 e_0) / (n - 1): piece k covers [k, k + 1) in
                         // u = (log2 e - lg0) * inv_dlg
    float inv_dlg;       // (n - 1) / (log2 e_{n-1} - log2 e_0)
    static constexpr int kMaxIter = 100;  // Newton steps at most
    // learned seed: predictions of the MLP on a grid over (ln E, |M|/E),
    // read by bilinear interpolation (the grid is filled by the MLP kernel)
    // (grid shape and spacing are compile-time constants: fewer scalar
    // registers in the sweeps)
    const float* seed;   // [kSeedG0][kSeedG1] or nullptr (plain solve)
    int32_t seed_output;             // 0: grid holds ln e; 1: the bracket fraction (E - e) E / |M|^2
    static constexpr double kSeedMinM2 = 2e-2;  // ln e seed only where (|M|/E)^2 > this
    // Newton stops when |de| <= kNewtonTol e and returns e - de.  The error of
    // that iterate is bounded by (max |g''| / (2 min g')) de^2 with
    // g' >= 1 - m^2 max p' and |g''| <= m^2 (2 max p'^2 / E + max |p''|): for
    // p' <= 1/3 and e |p''| <= 0.3 (the crossover table) it is below
    // 1e-14 e, far inside the 1e-12 the solve promises, one iteration sooner
    // than a stop at |de| <= 1e-12 e (which needs a confirming step).
    static constexpr double kNewtonTol = 1e-7;
    // g is a difference of O(E) terms, known to a few ulp of E: a correction
    // below kNewtonAbsTol E is rounding noise (for |M| -> E the root e << E is
    // only defined to that absolute level), and the iterate is accepted.
    static constexpr double kNewtonAbsTol = 1e-15;
    // The last first-guess piece this thread loaded (the thread's copy of the
    // EoS lives in registers).  Neighbouring cells of smooth flow look up the
    // same piece again and again; a wavefront whose lanes all guess the cached
    // piece takes it from registers and issues no loads.  The cache is keyed
    // by the first guess, so every lane evaluates the piece it would have
    // loaded: results do not depend on the cache's history.
    // The piece lives in a per-thread LDS slot (6 doubles, 256 apart), which the
    // kernel binds: kept in registers, the compiler copied it at every lookup.
    static constexpr int kCacheDoubles = 6 * 256;
    mutable int32_t ck = -1;
    mutable double* cl = nullptr;
    __device__ __forceinline__ void bind_cache(double* lds) const { cl = lds + threadIdx.x; }
    __device__ __forceinline__ void put(const double2& a, const double2& b, const double2& c) const
    {
        cl[0] = a.x; cl[256] = a.y; cl[512] = b.x; cl[768] = b.y; cl[1024] = c.x; cl[1280] = c.y;
    }
    __device__ __forceinline__ double cached_cubic(double e, double& p, double& dp) const
    {
        const double2 a = {cl[0], cl[256]}, b = {cl[512], cl[768]}, c = {cl[1024], cl[1280]};
        return cubic(e, a, b, c, p, dp);
    }

    // Piece k: records 3k .. 3k + 2 (the table is far below 4 GiB, so a 32-bit byte offset).
    __device__ __forceinline__ const double2* piece_ptr(int k) const
    {
        return reinterpret_cast<const double2*>(reinterpret_cast<const char*>(rec) + (uint32_t)k * 48u);
    }

    // Cubic of one piece at e: p and dp/de; returns t (the piece holds e for 0 <= t < 1).
    __device__ __forceinline__ static double cubic(double e, const double2& a, const double2& b, const double2& c,
                                                   double& p, double& dp)
    {
        const double t = (e - a.x) * a.y;
        p = fma(t, fma(t, fma(t, c.y, c.x), b.y), b.x);
        dp = a.y * fma(t, fma(t, 3.0 * c.y, 2.0 * c.x), b.y);
        return t;
    }

    // Lanes whose first-guess piece does not hold their argument (t outside [0, 1), or NaN).
    __device__ __forceinline__ static uint64_t outside(double t)
    {
        return lanes_where(!(t >= 0.0)) | lanes_where(!(t < 1.0));
    }

    // p(e) and dp/de (e >= 0).  On log-uniform nodes the piece comes from a
    // single-precision log2, which can be one piece off next to a node: the
    // cubic of the first guess is evaluated at once (so the piece's loads are
    // issued together), and lanes outside that piece's bounds redo it with the
    // right piece inside a wave-uniform branch.
    __device__ __forceinline__ int guess_piece(double e) const
    {
        float u = (__builtin_amdgcn_logf((float)e) - lg0) * inv_dlg;  // log2 (about 1 ulp)
        u = fminf(fmaxf(u, 0.0f), (float)n + 0.5f);                    // also maps NaN to 0
        return (int)u;                                                 // in [0, n]
    }

    // The piece of e found by stepping from piece k (piece j starts at the origin
    // of its record and ends at the next piece's), and its cubic.
    __device__ __forceinline__ void walk(double e, int k, double& p, double& dp) const
    {
        while (k > 0 && e < piece_ptr(k)[0].x) k--;
        while (k < n && e >= piece_ptr(k + 1)[0].x) k++;
        const double2* r = piece_ptr(k);
        cubic(e, r[0], r[1], r[2], p, dp);
    }

    __device__ __forceinline__ void eval(double e, double& p, double& dp) const
    {
        if (log_uniform) {
            const int k = guess_piece(e);
            uint64_t off;
            if (lanes_where(k != ck) != 0) {   // some lane needs another piece
                const double2* r = piece_ptr(k);
                const double2 a = r[0], b = r[1], c = r[2];
                put(a, b, c);
                ck = k;
                off = outside(cubic(e, a, b, c, p, dp));
            } else {
                off = outside(cached_cubic(e, p, dp));
            }
            if (off != 0) {
                if (lane_in(off)) walk(e, k, p, dp);
            }
        } else {
            int lo = 0, hi = n + 1;  // origin of piece lo <= e < origin of piece hi
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (piece_ptr(mid)[0].x <= e) lo = mid;
                else hi = mid;
            }
            const double2* r = piece_ptr(lo);
            cubic(e, r[0], r[1], r[2], p, dp);
        }
    }

    // eval of two arguments, with the loads of both first-guess pieces
    // issued before either is used (their latency overlaps).
    __device__ __forceinline__ void eval2(double eA, double eB, double& pA, double& dpA, double& pB,
                                          double& dpB) const
    {
        if (log_uniform) {
            const int kA = guess_piece(eA), kB = guess_piece(eB);
            uint64_t offA, offB;
            if ((lanes_where(kA != ck) | lanes_where(kB != ck)) != 0) {   // some lane needs another piece
                const double2* rA = piece_ptr(kA);
                const double2* rB = piece_ptr(kB);
                const double2 aA = rA[0], bA = rA[1], cA = rA[2];
                const double2 aB = rB[0], bB = rB[1], cB = rB[2];
                offA = outside(cubic(eA, aA, bA, cA, pA, dpA));
                offB = outside(cubic(eB, aB, bB, cB, pB, dpB));
                put(aB, bB, cB);
                ck = kB;
            } else {
                offA = outside(cached_cubic(eA, pA, dpA));
                offB = outside(cached_cubic(eB, pB, dpB));
            }
            if ((offA | offB) != 0) {
                if (lane_in(offA)) walk(eA, kA, pA, dpA);
                if (lane_in(offB)) walk(eB, kB, pB, dpB);
            }
        } else {
            eval(eA, pA, dpA);
            eval(eB, pB, dpB);
        }
    }

    // Root e of g on the bracket [lo, E], starting from e_start (inside the
    // bracket; E when M2 = 0), with p and dp/de at the root.  Newton steps that leave the
    // shrinking bracket are replaced by bisection.  At rest (M2 = 0) the root
    // is E and no iteration is counted.  On convergence p(e) is carried to the
    // accepted iterate to first order (the remainder is O(de^2) with
    // |de| <= 1e-7 e, below 1e-14 relative for the crossover table), so the
    // root costs no extra lookup.
    __device__ __forceinline__ double solve(double E, double M2, double lo, double e_start, double& p, double& dp,
                                            Counts& cnt) const
    {
        eval(e_start, p, dp);
        return newton(E, M2, lo, e_start, p, dp, cnt);
    }

    // The iterations of solve from e (p and dp/de at e given).
    __device__ __forceinline__ double newton(double E, double M2, double lo, double e, double& p, double& dp,
                                             Counts& cnt) const
    {
        if (__any(M2 != 0.0)) {  // wavefronts entirely at rest are done
            if (M2 != 0.0) {
                double hi = E;
                for (int it = 1;; it++) {
                    const double iw = Math<double>::rcp(E + p);
                    const double g = (e - E) + M2 * iw;
                    const double gp = 1.0 - M2 * dp * iw * iw;
                    const double de = g * Math<double>::rcp(gp);
                    double en = e - de;
                    cnt.iters += cnt.w;
                    // converged: accept the (small) Newton correction before any bracket test,
                    // which could otherwise reject an iterate sitting on the bracket edge
                    if (fabs(de) <= fmax(kNewtonTol * e, kNewtonAbsTol * E)) {
                        p = p - dp * de;
                        e = en;
                        break;
                    }
                    if (g > 0.0) hi = e;
                    else lo = e;
                    if (!(en > lo && en < hi)) en = 0.5 * (lo + hi);
                    e = en;
                    eval(e, p, dp);
                    if (it >= kMaxIter) break;  // iteration cap
                }
            }
        }
        return e;
    }

    // Start of a seeded solve: the guess e0 if it lies strictly inside the
    // bracket [lo, E], else the bracket midpoint (counted as a fallback).
    __device__ __forceinline__ static double seeded_start(double E, double lo, double e0, Counts& cnt)
    {
        if (e0 > lo && e0 < E) return e0;
        cnt.fallback += cnt.w;
        return 0.5 * (lo + E);
    }

    // Bilinear read of the seed grid at (ln E, m); q = |M|^2 / E.  Returns the guess e0.
    __device__ __forceinline__ double seed_guess(double E, double M2, double q) const
    {
        const float Ef = (float)E;
        const float lnE = __builtin_amdgcn_logf(Ef) * 0.69314718f;
        const float m = __builtin_amdgcn_sqrtf((float)M2) * __builtin_amdgcn_rcpf(Ef);
        constexpr float lnE0 = (float)kSeedLnLo;
        constexpr float inv_dlnE = (float)(1.0 / ((kSeedLnHi - kSeedLnLo) / (kSeedG0 - 1)));
        float u = (lnE - lnE0) * inv_dlnE;
        float v = m * (float)(kSeedG1 - 1);
        // clamps also map NaN to 0 (fmaxf returns the other operand)
        u = fminf(fmaxf(u, 0.0f), (float)(kSeedG0 - 1) - 1e-3f);
        v = fminf(fmaxf(v, 0.0f), (float)(kSeedG1 - 1) - 1e-3f);
        const int i = (int)u, j = (int)v;
        const float fu = u - (float)i, fv = v - (float)j;
        const float* r0 = seed + i * kSeedG1 + j;
        const float* r1 = r0 + kSeedG1;
        const float y = (1.0f - fu) * ((1.0f - fv) * r0[0] + fv * r0[1]) + fu * ((1.0f - fv) * r1[0] + fv * r1[1]);
        if (seed_output == 1) return E - (double)y * q;
        return (double)__expf(y);
    }

    // e, p and dp/de of a state with |M|^2 = M2 (E > 0, |M| < E).
    __device__ __forceinline__ double recover(double E, double M2, double& p, double& dp, Counts& cnt) const
    {
        double lo, e_start;
        start(E, M2, lo, e_start, cnt);
        return solve(E, M2, lo, e_start, p, dp, cnt);
    }

    // Bracket [lo, E] of the root and the start of the solve: E at rest,
    // else the seed's guess (see seeded_start) or the bracket midpoint.
    __device__ __forceinline__ void start(double E, double M2, double& lo, double& e_start, Counts& cnt) const
    {
        lo = E;
        e_start = E;
        if (__any(M2 != 0.0)) {  // wavefronts entirely at rest need no bracket
            const double q = M2 * Math<double>::rcp(E);
            lo = E - q;
            e_start = 0.5 * (lo + E);
            // A guess of ln e carries an error of about 1e-4 to 1e-2 relative; the
            // bracket midpoint is off by about m^2 E / 4.  The guess saves a Newton
            // step only where m^2 > kSeedMinM2 (on the crossover workload a threshold
            // of 1e-3 saved no more iterations than 2e-2), so that seed is consulted
            // only there (wavefronts without such a state skip the lookup).  A guess
            // of the bracket fraction is scaled by the bracket and consulted wherever
            // |M| > 0.
            if (seed) {
                const bool wide = q > (seed_output == 1 ? 0.0 : kSeedMinM2 * E);
                if (__any(wide)) {
                    if (wide) e_start = seeded_start(E, lo, seed_guess(E, M2, q), cnt);
                }
            }
        }
    }

    __device__ __forceinline__ bool fixup(double& E, double& Mx, double& My, double& Mz, double& M2,
                                          Counts& cnt) const
    {
        if (!((E > 0.0) & (E <= big_value<double>()) & (M2 <= big_value<double>()))) {
            cnt.bad += cnt.w;
            return false;
        }
        const double Mlim = mmax<double>() * E;
        if (M2 > Mlim * Mlim) {
            const double s = Mlim / Math<double>::sqrt_safe(M2);
            Mx = Mx * s; My = My * s; Mz = Mz * s;
            M2 = Mx * Mx + My * My + Mz * Mz;
            cnt.floor_ += cnt.w;
        }
        return true;
    }

    // Guards for every lane of the wavefront at once: states that need one
    // are fixed (or replaced by a harmless state at rest and flagged) inside a
    // wave-uniform branch, so the solve below runs once for all lanes.
    // Near-vacuum states (E below tiny_value) are scaled up by up_scale (the
    // table is linear there, so con2prim is invariant): their lanes are
    // returned in *scaled, whose fluxes the caller scales back.
    __device__ __forceinline__ bool guard(double& E, double& Mx, double& My, double& Mz, double& M2,
                                          Counts& cnt, uint64_t& scaled) const
    {
        const double Mlim = mmax<double>() * E;
        const uint64_t bad = lanes_where(!(E >= tiny_value<double>())) | lanes_where(!(E <= big_value<double>())) |
                             lanes_where(!(M2 <= Mlim * Mlim));
        bool live = true;
        scaled = 0;
        if (bad != 0) {
            const bool small = (E > 0.0) & (E < tiny_value<double>());
            scaled = lanes_where(small);
            if (lane_in(bad)) {
                if (small) {
                    E = E * up_scale<double>(); Mx = Mx * up_scale<double>();
                    My = My * up_scale<double>(); Mz = Mz * up_scale<double>();
                    M2 = Mx * Mx + My * My + Mz * Mz;
                }
                live = fixup(E, Mx, My, Mz, M2, cnt);
                if (!live) {
                    E = 1.0; Mx = 0.0; My = 0.0; Mz = 0.0; M2 = 0.0;
                }
            }
        }
        return live;
    }

    // Fluxes of the scaled lanes back to the state's scale.
    __device__ __forceinline__ static void unscale(uint64_t scaled, double F[4])
    {
        if (scaled != 0) {
            if (lane_in(scaled)) {
#pragma unroll
                for (int c = 0; c < 4; c++) F[c] = F[c] * down_scale<double>();
            }
        }
    }

    // Flux from the recovered pressure.
    template <int D>
    __device__ __forceinline__ static void assemble(double E, double Mx, double My, double Mz, double p, bool live,
                                                    double F[4])
    {
        const double MD = (D == 0) ? Mx : ((D == 1) ? My : Mz);
        const double vD = MD * Math<double>::rcp(E + p);
        F[0] = MD;  // (E + p) v_D
        F[1] = Mx * vD;
        F[2] = My * vD;
        F[3] = Mz * vD;
        // a replaced state is at rest (M = 0, so vD = 0): only the pressure term is non-zero
        F[1 + D] = live ? F[1 + D] + p : 0.0;
    }

    template <int D, int NC = 4>
    __device__ __forceinline__ void flux(const double u[], double F[], Counts& cnt) const
    {
        static_assert(NC == 4, "the tabulated EoS carries no charge");
        double E = u[0], Mx = u[1], My = u[2], Mz = u[3];
        double M2 = Mx * Mx + My * My + Mz * Mz;
        uint64_t scaled;
        const bool live = guard(E, Mx, My, Mz, M2, cnt, scaled);
        double p, dp;
        recover(E, M2, p, dp, cnt);
        assemble<D>(E, Mx, My, Mz, p, live, F);
        unscale(scaled, F);
    }
    // Flux of a state formed from the last pair (the solve starts as in flux).
    template <int D, int NC = 4>
    __device__ __forceinline__ void flux_near(const double u[], double F[], Counts& cnt) const
    {
        flux<D, NC>(u, F, cnt);
    }

    // Fluxes of two independent states, computed as flux() does but with the
    // first table lookups of both issued together (eval2): in the sweeps the
    // lookups are L2 hits whose latency would otherwise be paid twice.
    // (CHAIN: see EosGamma::flux2; the table solves start as in flux.)
    template <int D, int NC = 4, bool CHAIN = false>
    __device__ __forceinline__ void flux2(const double uA[], const double uB[], double FA[], double FB[],
                                          Counts& cnt) const
    {
        static_assert(NC == 4, "the tabulated EoS carries no charge");
        double EA = uA[0], MxA = uA[1], MyA = uA[2], MzA = uA[3];
        double EB = uB[0], MxB = uB[1], MyB = uB[2], MzB = uB[3];
        double M2A = MxA * MxA + MyA * MyA + MzA * MzA;
        double M2B = MxB * MxB + MyB * MyB + MzB * MzB;
        uint64_t scA, scB;
        const bool liveA = guard(EA, MxA, MyA, MzA, M2A, cnt, scA);
        const bool liveB = guard(EB, MxB, MyB, MzB, M2B, cnt, scB);
        double loA, eA, loB, eB;
        start(EA, M2A, loA, eA, cnt);
        start(EB, M2B, loB, eB, cnt);
        double pA, dpA, pB, dpB;
        eval2(eA, eB, pA, dpA, pB, dpB);
        newton(EA, M2A, loA, eA, pA, dpA, cnt);
        newton(EB, M2B, loB, eB, pB, dpB, cnt);
        assemble<D>(EA, MxA, MyA, MzA, pA, liveA, FA);
        assemble<D>(EB, MxB, MyB, MzB, pB, liveB, FB);
        unscale(scA, FA);
        unscale(scB, FB);
    }

    __device__ __forceinline__ void prim(const double u[], double& e, double& p, double v[3], double& cs2,
                                         Counts& cnt) const
    {
        const bool small = (u[0] > 0.0) & (u[0] < tiny_value<double>());
        const double sc = small ? up_scale<double>() : 1.0;
        double E = u[0] * sc, Mx = u[1] * sc, My = u[2] * sc, Mz = u[3] * sc;
        double M2 = Mx * Mx + My * My + Mz * Mz;
        if (!fixup(E, Mx, My, Mz, M2, cnt)) {
            e = 0.0; p = 0.0; v[0] = 0.0; v[1] = 0.0; v[2] = 0.0; cs2 = 0.0;
            return;
        }
        double dp;
        e = recover(E, M2, p, dp, cnt);
        const double iw = Math<double>::rcp(E + p);
        v[0] = Mx * iw; v[1] = My * iw; v[2] = Mz * iw;
        cs2 = dp;
        if (small) {
            e = e * down_scale<double>();
            p = p * down_scale<double>();
        }
    }
};


// ---------------------------------------------------------------------------
// Ideal gas with the conserved charge (Sec. 2.1 closure p = p(e, n)):
// p = (gamma - 1) max(e - n, 0), n the rest-frame charge density.  FP64, 5
// components only.
//
// con2prim (Sec. 2.6): with e = E - |M|^2 / (E + p) and
// n = R sqrt(1 - |M|^2 / (E + p)^2) the fixed point for v is the root of
//   f(p) = (gamma - 1)(e(p) - n(p)) - p,
// which decreases in p (for gamma <= 2): f' = (gamma - 1) v^2 (1 - R W / (E + p)) - 1.
// If f(0) <= 0 the gas is cold (p = 0, v = M / E).  Otherwise safeguarded
// Newton on [0, (gamma - 1) E] from p = f(0), or from a neighbouring state's
// pressure in the sweeps (flux2, flux_near): a step leaving the bracket
// (which shrinks with the sign of f) is replaced by bisection; the solve stops
// when the correction is below 1e-10 (E + p) and accepts it (quadratic
// convergence leaves an error far below the rounding of f).
// ---------------------------------------------------------------------------
struct EosGamma {
    static constexpr int kWaves = 3;            // five components: more live state per interface
    static constexpr bool kLoadLAhead = false;
    static constexpr int kCacheDoubles = 1;  // no lookup cache
    __device__ __forceinline__ void bind_cache(double*) const {}
    static constexpr int kMaxIter = 60;
    static constexpr double kTol = 1e-10;
    double gm1;    // gamma - 1
    double gam;    // gamma

    static EosGamma make(double gamma)
    {
        EosGamma g;
        g.gam = gamma;
        g.gm1 = gamma - 1.0;
        return g;
    }

    // f(p) and f'(p); iw = 1 / (E + p) out.  f' takes W = 1/sqrt(1 - v^2) from
    // the square root's own step (about 1e-15 relative), which the Newton step
    // tolerates: only f decides the root.
    __device__ __forceinline__ void residual(double E, double M2, double R, double p, double& f, double& fp,
                                             double& iw) const
    {
        iw = Math<double>::rcp(E + p);
        const double v2 = M2 * iw * iw;
        double W;
        const double sq = Math<double>::sqrt_rsq(1.0 - v2, W);   // 1 / W, and W
        const double e = E - M2 * iw;
        f = gm1 * (e - R * sq) - p;
        fp = gm1 * v2 * (1.0 - R * iw * W) - 1.0;
    }

    // Pressure of a live state (E > 0, |M| < E, R >= 0).  The iteration starts
    // from p0 where 0 < p0 < (gamma - 1) E (a neighbouring state's pressure),
    // else from min(f(0), (gamma - 1) E) once f(0) > 0 has ruled out cold gas.
    // STEP_FIRST takes the first step from p0 before the cold-gas test (which
    // a converged positive step makes unnecessary); the x sweep, whose
    // neighbouring states differ more, runs the test first (it measured faster).
    // iwp returns 1 / (E + p) for the returned p.  After an accepted step it is
    // the last residual's 1 / (E + p_k) carried to p = p_k - d to first order,
    // iw (1 + d iw): d iw <= kTol, so the remainder (d iw)^2 is below 1e-20.
    template <bool STEP_FIRST = true>
    __device__ __forceinline__ double pressure(double E, double M2, double R, Counts& cnt, double& iwp,
                                               double p0 = -1.0) const
    {
        if (M2 == 0.0) {
            const double p = gm1 * fmax(E - R, 0.0);
            iwp = Math<double>::rcp(E + p);
            return p;
        }
        double f, fp, iw;
        double lo = 0.0, hi = gm1 * E;
        double p;
        if (STEP_FIRST && p0 > 0.0 && p0 < hi) {
            // The first Newton step from p0.  A step accepted at a positive
            // p needs no cold-gas test: f decreases, so f(0) > f(root) = 0.
            residual(E, M2, R, p0, f, fp, iw);
            const double dp = f * __builtin_amdgcn_rcp(fp);
            p = p0 - dp;
            cnt.iters += cnt.w;
            if (fabs(dp) <= kTol * (E + p0) && p > 0.0) {
                iwp = fma(iw * dp, iw, iw);
                return p;
            }
            if (f > 0.0) lo = p0;
            else hi = p0;
            double f0, fp0, iw0;
            residual(E, M2, R, 0.0, f0, fp0, iw0);
            if (!(f0 > 0.0)) {   // cold gas
                iwp = iw0;
                return 0.0;
            }
            if (!(p > lo && p < hi)) p = 0.5 * (lo + hi);
        } else {
            residual(E, M2, R, 0.0, f, fp, iw);
            if (!(f > 0.0)) {   // cold gas
                iwp = iw;
                return 0.0;
            }
            p = (p0 > 0.0 && p0 < hi) ? p0 : fmin(f, hi);
        }
        for (int it = 1;; it++) {
            residual(E, M2, R, p, f, fp, iw);
            // fp < 0 (about -1).  The hardware reciprocal (5e-8 relative) suffices: a
            // step accepted at |dp| <= kTol (E + p) then errs by below 1e-17 (E + p).
            const double dp = f * __builtin_amdgcn_rcp(fp);
            double pn = p - dp;
            cnt.iters += cnt.w;
            if (fabs(dp) <= kTol * (E + p)) {
                const double pr = fmax(pn, 0.0);
                iwp = fma(iw * (p - pr), iw, iw);
                return pr;
            }
            if (f > 0.0) lo = p;
            else hi = p;
            if (!(pn > lo && pn < hi)) pn = 0.5 * (lo + hi);
            p = pn;
            if (it >= kMaxIter) {
                iwp = Math<double>::rcp(E + p);
                return p;
            }
        }
    }

    // Guards: E <= 0, a non-finite component or R < 0 -> bad (the zero state:
    // zero flux); |M| above (1 - 1e-12) E is scaled to that bound.  Returns false
    // for the zero state.
    __device__ __forceinline__ bool fixup(double& E, double& Mx, double& My, double& Mz, double& M2, double R,
                                          Counts& cnt) const
    {
        if (!((E > 0.0) & (E <= big_value<double>()) & (M2 <= big_value<double>()) & (R >= 0.0) &
              (R <= big_value<double>()))) {
            cnt.bad += cnt.w;
            return false;
        }
        const double Mlim = mmax<double>() * E;
        if (M2 > Mlim * Mlim) {
            const double s = Mlim / Math<double>::sqrt_safe(M2);
            Mx = Mx * s; My = My * s; Mz = Mz * s;
            M2 = Mx * Mx + My * My + Mz * Mz;
            cnt.floor_ += cnt.w;
        }
        return true;
    }

    // Flux of u; the pressure's iteration starts from p0 (see pressure).
    // Returns the pressure, or -1 for a state evaluated scaled or zeroed.
    template <int D, int NC = 5>
    __device__ __forceinline__ double flux_from(const double u[], double F[], Counts& cnt, double p0) const
    {
        static_assert(NC == 5, "the ideal gas needs the charge");
        double E = u[0], Mx = u[1], My = u[2], Mz = u[3], R = u[4];
        double M2 = Mx * Mx + My * My + Mz * Mz;
        // The guards run only in wavefronts holding a state that needs one (the
        // vote covers every case fixup handles): near-vacuum states are
        // evaluated scaled up (con2prim of the ideal gas is scale invariant).
        const double Mlim = mmax<double>() * E;
        const uint64_t bad = lanes_where(!(E >= tiny_value<double>())) | lanes_where(!(E <= big_value<double>())) |
                             lanes_where(!(M2 <= Mlim * Mlim)) | lanes_where(!(M2 <= big_value<double>())) |
                             lanes_where(!(R >= 0.0)) | lanes_where(!(R <= big_value<double>()));
        bool small = false, live = true;
        if (bad != 0) {
            if (lane_in(bad)) {
                small = (E > 0.0) & (E < tiny_value<double>());
                if (small) {
                    E = E * up_scale<double>(); Mx = Mx * up_scale<double>(); My = My * up_scale<double>();
                    Mz = Mz * up_scale<double>(); R = R * up_scale<double>();
                    M2 = Mx * Mx + My * My + Mz * Mz;
                }
                live = fixup(E, Mx, My, Mz, M2, R, cnt);
            }
        }
        if (!live) {
#pragma unroll
            for (int c = 0; c < 5; c++) F[c] = 0.0;
            return -1.0;
        }
        double iw;
        const double p = pressure<(D > 0)>(E, M2, R, cnt, iw, small ? -1.0 : p0);
        const double MD = (D == 0) ? Mx : ((D == 1) ? My : Mz);
        const double vD = MD * iw;
        F[0] = MD;  // (E + p) v_D
        F[1] = Mx * vD;
        F[2] = My * vD;
        F[3] = Mz * vD;
        F[1 + D] = F[1 + D] + p;
        F[4] = R * vD;
        if (small) {
#pragma unroll
            for (int c = 0; c < 5; c++) F[c] = F[c] * down_scale<double>();
            return -1.0;
        }
        return p;
    }

    template <int D, int NC = 5>
    __device__ __forceinline__ void flux(const double u[], double F[], Counts& cnt) const
    {
        flux_from<D, NC>(u, F, cnt, -1.0);
    }

    // The two states of a pair (the faces of one cell, or the two sides of an
    // interface) are close where the flow is smooth: B's iteration starts
    // from A's pressure.  The mean of the two pressures is kept for the
    // state that the next flux_near call forms from the pair.  With CHAIN,
    // A's iteration starts from the previous pair's A: the pairs of a MUSTA
    // solve follow the Hancock pair of the interface's right-hand cell, whose
    // A is that cell's left face, at the same interface; each later stage's A
    // is the predictor's update of the one before.  The sweeps evaluate that
    // Hancock pair right before the interface's MUSTA solve, so every start
    // comes from the same interface and results do not depend on the work
    // decomposition.
    mutable double p_pair = -1.0;
    mutable double p_first = -1.0;
    template <int D, int NC = 5, bool CHAIN = false>
    __device__ __forceinline__ void flux2(const double uA[], const double uB[], double FA[], double FB[],
                                          Counts& cnt) const
    {
        const double pA = flux_from<D, NC>(uA, FA, cnt, CHAIN ? p_first : -1.0);
        const double pB = flux_from<D, NC>(uB, FB, cnt, pA);
        p_pair = (pA > 0.0 && pB > 0.0) ? 0.5 * (pA + pB) : -1.0;
        p_first = pA;
    }
    // Flux of a state formed from the last flux2 pair (the Richtmyer state of a
    // MUSTA stage): its iteration starts from the pair's mean pressure.  The
    // start is used once, so the result depends only on that pair.
    template <int D, int NC = 5>
    __device__ __forceinline__ void flux_near(const double u[], double F[], Counts& cnt) const
    {
        flux_from<D, NC>(u, F, cnt, p_pair);
        p_pair = -1.0;
    }

    // cs2 = gamma p / (e + p) (0 for cold gas).
    __device__ __forceinline__ void prim(const double u[], double& e, double& p, double v[3], double& cs2,
                                         Counts& cnt) const
    {
        const bool small = (u[0] > 0.0) & (u[0] < tiny_value<double>());
        const double sc = small ? up_scale<double>() : 1.0;
        double E = u[0] * sc, Mx = u[1] * sc, My = u[2] * sc, Mz = u[3] * sc;
        const double R = u[4] * sc;
        double M2 = Mx * Mx + My * My + Mz * Mz;
        if (!fixup(E, Mx, My, Mz, M2, R, cnt)) {
            e = 0.0; p = 0.0; v[0] = 0.0; v[1] = 0.0; v[2] = 0.0; cs2 = 0.0;
            return;
        }
        double iw;
        p = pressure(E, M2, R, cnt, iw);
        v[0] = Mx * iw; v[1] = My * iw; v[2] = Mz * iw;
        e = E - M2 * iw;
        cs2 = p > 0.0 ? gam * p * Math<double>::rcp(e + p) : 0.0;
        if (small) {
            e = e * down_scale<double>();
            p = p * down_scale<double>();
        }
    }
};


// ---------------------------------------------------------------------------
// Slope limiters (Sec. 2.5) in the two-argument form phi(a, b) = xi(b/a) a,
// a = U_i - U_{i-1}, b = U_{i+1} - U_i.  For the symmetric limiters of the
// paper the left and right face slopes coincide, U^{L,R} = U -/+ phi / 2.
// "Same sign" = both non-zero with equal signs (no product, which could
// underflow).
// ---------------------------------------------------------------------------
template <int LIM, typename T>
__device__ __forceinline__ T limiter(T a, T b)
{
    if constexpr (LIM == LIM_NONE) {
        return T(0.5) * (a + b);
    } else if constexpr (LIM == LIM_VANALBADA) {
        const T den = a * a + b * b;
        return (den > T(0)) ? (a * b * (a + b)) / den : T(0);
    } else if constexpr (LIM == LIM_VANLEER) {
        // 2ab / (a + b) = 2|a||b| / (|a| + |b|) with the sign of a, for equal signs
        const bool same = (fmin(a, b) > T(0)) | (fmax(a, b) < T(0));
        const T aa = fabs(a), bb = fabs(b);
        const T m = Math<T>::div(T(2) * aa * bb, aa + bb);
        return same ? copysign(m, a) : T(0);
    } else {
        // With s = sign(a): s b < 0 when the signs differ, and s b = 0 or
        // |a| = 0 when one difference vanishes, so max(0, min(..)) is the
        // "same sign" test; the result carries the sign s.
        const T s = copysign(T(1), a);
        const T aa = fabs(a);
        const T sb = s * b;
        T m;
        if constexpr (LIM == LIM_MINMOD) {
            m = fmin(aa, sb);
        } else if constexpr (LIM == LIM_SUPERBEE) {
            m = fmax(fmin(T(2) * sb, aa), fmin(sb, T(2) * aa));
        } else {  // LIM_MC
            m = fmin(T(2) * fmin(aa, sb), T(0.5) * (aa + sb));
        }
        return s * fmax(m, T(0));
    }
}

// phi(a, b) / 2, the offset of the face states from the cell value.  For MC
// the factor is folded into the limiter's terms (exact: power-of-two scaling
// commutes with min and max), saving a multiply.
template <int LIM, typename T>
__device__ __forceinline__ T half_slope(T a, T b)
{
    if constexpr (LIM == LIM_MC) {
        const T s = copysign(T(1), a);
        const T aa = fabs(a);
        const T sb = s * b;
        return s * fmax(fmin(fmin(aa, sb), T(0.25) * (aa + sb)), T(0));
    } else {
        return T(0.5) * limiter<LIM>(a, b);
    }
}

// ---------------------------------------------------------------------------
// MUSCL reconstruction + Hancock half step for one cell along axis D
// (Sec. 2.4: piecewise-linear cell profile, faces U^L = U - Delta/2,
// U^R = U + Delta/2, both advanced by (dt/2dx)(F(U^L) - F(U^R))).
// ---------------------------------------------------------------------------
// PAIRED: evaluate the two face fluxes with Eos::flux2 (overlapped table
// lookups; more registers), else one after the other.  CHAIN: the pair
// continues the previous pair's interface (Eos::flux2).
template <int D, typename T, class Eos, bool PAIRED, int NC = 4, bool CHAIN = false>
__device__ __forceinline__ void flux_pair(const Eos& eos, const T uA[], const T uB[], T FA[], T FB[], Counts& cnt)
{
    if constexpr (PAIRED) {
        eos.template flux2<D, NC, CHAIN>(uA, uB, FA, FB, cnt);
    } else {
        eos.template flux<D, NC>(uA, FA, cnt);
        eos.template flux<D, NC>(uB, FB, cnt);
    }
}

// NC: conserved components (4, or 5 with the charge R).
template <int D, int LIM, bool PAIRED, int NC = 4, typename T, class Eos>
__device__ __forceinline__ void hancock(const T um[], const T u0[], const T up[], T half_lam,
                                        T ULt[], T URt[], const Eos& eos, Counts& cnt)
{
    T UL[NC], UR[NC], FL[NC], FR[NC];
#pragma unroll
    for (int c = 0; c < NC; c++) {
        const T hs = half_slope<LIM>(u0[c] - um[c], up[c] - u0[c]);
        UL[c] = u0[c] - hs;
        UR[c] = u0[c] + hs;
    }
    flux_pair<D, T, Eos, PAIRED, NC>(eos, UL, UR, FL, FR, cnt);
#pragma unroll
    for (int c = 0; c < NC; c++) {
        const T dF = FL[c] - FR[c];   // both faces move by (dt/2dx) dF
        ULt[c] = fma(half_lam, dF, UL[c]);
        URt[c] = fma(half_lam, dF, UR[c]);
    }
}

// Faces of one cell under the unsplit Hancock reading (the ablation of the
// per-axis step): U^{L,R} = U -/+ phi / 2, both moved by the cell's
// correction d, which sums the three axes' Hancock terms and is computed once
// per stage for the whole grid (component c of a cell at dl[c * dl_n]).
template <typename T>
__device__ __forceinline__ void load_dl(const T* dl, int64_t dl_n, T d[4])
{
#pragma unroll
    for (int c = 0; c < 4; c++) d[c] = dl[c * dl_n];
}

template <int LIM, typename T>
__device__ __forceinline__ void unsplit_faces(const T um[4], const T u0[4], const T up[4], const T d[4], T ULt[4],
                                              T URt[4])
{
#pragma unroll
    for (int c = 0; c < 4; c++) {
        const T hs = half_slope<LIM>(u0[c] - um[c], up[c] - u0[c]);
        ULt[c] = (u0[c] - hs) + d[c];
        URt[c] = (u0[c] + hs) + d[c];
    }
}

// ---------------------------------------------------------------------------
// MUSTA-FORCE flux at one interface (Sec. 2.4): k stages of the FORCE flux
//   F_lw = F(1/2 (U_L + U_R) - alpha dt/(2dx) (F_R - F_L))     (Richtmyer)
//   F_lf = 1/2 (F_L + F_R) - dx/(2 alpha dt) (U_R - U_L)
//   F    = 1/2 (F_lw + F_lf)
// with the local predictor U_L -= dt/dx (F - F_L), U_R -= dt/dx (F_R - F)
// between stages.  UL and UR are consumed.  Returns G = 2 F = F_lw + F_lf
// (the average's factor 1/2 is exact and is applied with the flux
// difference, where it folds into the 1/dx factor).
// ---------------------------------------------------------------------------
template <int D, bool PAIRED, int NC = 4, typename T, class Eos>
__device__ __forceinline__ void musta(T UL[], T UR[], int k, const AxisConst<T>& ac, T G[],
                                      const Eos& eos, Counts& cnt)
{
    for (int l = 1;; l++) {
        T FL[NC], FR[NC], Us[NC], Flw[NC];
        flux_pair<D, T, Eos, PAIRED, NC, true>(eos, UL, UR, FL, FR, cnt);
#pragma unroll
        for (int c = 0; c < NC; c++) Us[c] = T(0.5) * (UL[c] + UR[c]) - ac.half_alam * (FR[c] - FL[c]);
        eos.template flux_near<D, NC>(Us, Flw, cnt);
#pragma unroll
        for (int c = 0; c < NC; c++)
            G[c] = fma(T(0.5), FL[c] + FR[c], fma(-ac.inv_2alam, UR[c] - UL[c], Flw[c]));
        if (l >= k) break;
#pragma unroll
        for (int c = 0; c < NC; c++) {
            UL[c] = UL[c] - ac.lam * fma(T(0.5), G[c], -FL[c]);   // F - F_L
            UR[c] = UR[c] - ac.lam * fma(T(-0.5), G[c], FR[c]);   // F_R - F
        }
    }
}

// Largest |characteristic speed| of a primitive state over the three axes:
// lambda_pm = [v_d (1 - cs2) +- cs sqrt((1 - v^2)(1 - v_d^2 - (v^2 - v_d^2) cs2))] / (1 - v^2 cs2).
// Along axis d the larger magnitude has the sign of v_d and equals
// (|v_d| B + sqrt(cs2 (1 - v^2)(A - v_d^2 B))) / A with A = 1 - v^2 cs2 and
// B = 1 - cs2; it increases with |v_d| (its derivative is positive for
// v_d^2 < 1), so the maximum over the axes is taken on the axis of largest
// |v_d| and one square root suffices.
template <typename T>
__device__ __forceinline__ T max_speed(const T v[3], T cs2)
{
    const T v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    const T vm = fmax(fabs(v[0]), fmax(fabs(v[1]), fabs(v[2])));
    const T A = T(1) - v2 * cs2;
    const T B = T(1) - cs2;
    T rad = cs2 * ((T(1) - v2) * (A - vm * vm * B));
    rad = rad > T(0) ? rad : T(0);
    return (vm * B + Math<T>::sqrt0(rad)) * Math<T>::rcp(A);
}

}  // namespace mf
