/*
 * mf_oracle.c -- plain FP64 CPU oracle of one MUSTA-FORCE time step of ideal
 * relativistic hydrodynamics (Porter-Sobieraj et al., "A MUSTA-FORCE
 * algorithm for solving partial differential equations of relativistic
 * hydrodynamics", arXiv:1510.06340).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * HIP library is checked against.  Only the tests, the smoke check and the
 * bench's CPU-baseline leg load it; the GPU library neither links nor calls
 * it, and the two share no code.
 *
 * It is written to be read against the paper, not to be fast: every step is
 * taken in the paper's order, on explicit ghost-padded lines, in IEEE double
 * precision with no FMA contraction (build with -ffp-contract=off).  OpenMP
 * only distributes independent grid lines; a cell's arithmetic does not
 * depend on the thread count.
 *
 * Readings of points the paper leaves open (each is marked READING below):
 *  - Lax-Wendroff argument: Richtmyer form, the half-step state is
 *    1/2(UL+UR) - alpha*dt/(2dx) (F(UR) - F(UL)) (Sec. 2.4, LW flux equation;
 *    the printed U-difference is dimensionally inconsistent with the LF term).
 *  - MUSTA predictor uses dt/dx (as printed), FORCE uses alpha*dt/dx.
 *  - k stages = k FORCE evaluations and k-1 predictor updates.
 *  - Face states: interface i+1/2 takes U_L = Ut^R_i and U_R = Ut^L_{i+1}.
 *  - Hancock half step: only the sweep axis' flux difference (dimensionally
 *    split reading of the Sec. 2.4 MUSCL-Hancock equations).
 *  - Limiter in two-argument form phi(a,b) = xi(b/a) a, equal to the paper's
 *    ratio form for symmetric limiters (Sec. 2.5) and defined at a = 0.
 *  - Boundaries: two ghost layers, outflow = copy of the edge cell,
 *    periodic = wrap.
 *  - Unphysical states: E <= 0 or non-finite -> counted, zero flux;
 *    |M| > (1 - 1e-12) E -> M scaled to that bound for the evaluation only,
 *    counted.
 * Two options give the alternative readings for ablations: predictor_alpha
 * (alpha*dt/dx in the MUSTA predictor) and unsplit_hancock (one Hancock
 * correction per cell from all three axes, added to all six faces).
 *
 * Parity unpinned: the paper prints no values that fix these readings (or
 * the combination of them); they are pinned only through invariants
 * (uniform states, mirror and planar symmetry, conservation) and exact
 * solutions (the shock tube and the Hubble-like expansion).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

enum { LIM_NONE = 0, LIM_MINMOD, LIM_SUPERBEE, LIM_MC, LIM_VANLEER, LIM_VANALBADA };
enum { BC_OUTFLOW = 0, BC_PERIODIC = 1 };
enum { EOS_IDEAL = 0, EOS_TABLE = 1, EOS_GAMMA = 2 };
#define NCMAX 5 /* E, Mx, My, Mz and the conserved charge R */

#define ORA_MMAX (1.0 - 1e-12) /* largest admitted |M|/E */

typedef struct {
    int32_t n[3];      /* cells along x, y, z */
    int32_t bc[3];     /* BC_OUTFLOW or BC_PERIODIC per axis */
    double dx[3];      /* cell sizes */
    double xlo[3];     /* lower box corner; cell centres at xlo + (i+1/2) dx */
    int32_t limiter;
    int32_t k;         /* MUSTA stages (>= 1) */
    int32_t rk;        /* Runge-Kutta order, 2 or 3 */
    double alpha;      /* FORCE coefficient, 3 in three dimensions */
    int32_t eos;       /* EOS_IDEAL: p = cs2 e; EOS_TABLE: monotone cubic table */
    double cs2;
    int32_t ntab;
    const double* etab; /* strictly increasing energy densities */
    const double* ptab; /* pressures at the nodes */
    const double* mtab; /* node slopes dp/de of the interpolant (ora_pchip_slopes) */
    int32_t jet;        /* 1: add the moving point-jet source */
    double jet_x0[3];   /* jet position at t = 0 */
    double jet_v;       /* jet speed along +x */
    double jet_dedx;    /* deposited dE/dx */
    double jet_sigma;   /* Gaussian width of the deposition */
    int32_t predictor_alpha; /* 1: alpha dt/dx in the MUSTA predictor (the alternative
                                reading of Sec. 2.4; 0: dt/dx as printed) */
    int32_t unsplit_hancock; /* 1: one Hancock correction per cell from all three axes,
                                added to all six faces (the alternative reading of the
                                multi-dimensional MUSCL-Hancock step, Sec. 2.4); 0: per axis */
    int32_t charge;     /* 1: a fifth conserved component, the charge R = n gamma (Sec. 2.1),
                           with flux R v_d; 0: U = (E, Mx, My, Mz) */
    double gamma;       /* EOS_GAMMA: p = (gamma - 1) (e - n), floored at 0 (needs charge) */
} ora_params;

/* Conserved components per cell. */
static int ncomp(const ora_params* P) { return P->charge ? 5 : 4; }

typedef struct {
    int64_t n_floor;  /* |M| clamped to (1-1e-12) E */
    int64_t n_bad;    /* E <= 0 or non-finite */
    int64_t n_iter;   /* root-finder iterations (table EoS) */
    int64_t n_calls;  /* con2prim evaluations */
} ora_counters;

/* ---------------------------------------------------------------------- */
/* Equation of state                                                       */
/* ---------------------------------------------------------------------- */

/* Monotone cubic Hermite node slopes (Fritsch & Carlson 1980; interior
 * weights of Fritsch & Butland 1984; three-point one-sided end slopes with
 * the monotonicity clamp). */
void ora_pchip_slopes(int32_t n, const double* x, const double* y, double* m)
{
    if (n < 2) { if (n == 1) m[0] = 0.0; return; }
    double* h = (double*)malloc(sizeof(double) * (size_t)(n - 1));
    double* d = (double*)malloc(sizeof(double) * (size_t)(n - 1));
    for (int i = 0; i < n - 1; i++) {
        h[i] = x[i + 1] - x[i];
        d[i] = (y[i + 1] - y[i]) / h[i];
    }
    if (n == 2) { m[0] = d[0]; m[1] = d[0]; free(h); free(d); return; }
    for (int i = 1; i < n - 1; i++) {
        if (d[i - 1] == 0.0 || d[i] == 0.0 || (d[i - 1] > 0.0) != (d[i] > 0.0)) {
            m[i] = 0.0;
        } else {
            double w1 = 2.0 * h[i] + h[i - 1];
            double w2 = h[i] + 2.0 * h[i - 1];
            m[i] = (w1 + w2) / (w1 / d[i - 1] + w2 / d[i]);
        }
    }
    /* end slopes */
    for (int end = 0; end < 2; end++) {
        double h0, h1, d0, d1;
        int idx;
        if (end == 0) { h0 = h[0]; h1 = h[1]; d0 = d[0]; d1 = d[1]; idx = 0; }
        else { h0 = h[n - 2]; h1 = h[n - 3]; d0 = d[n - 2]; d1 = d[n - 3]; idx = n - 1; }
        double s = ((2.0 * h0 + h1) * d0 - h0 * d1) / (h0 + h1);
        if ((s > 0.0) != (d0 > 0.0) || s == 0.0 || d0 == 0.0) s = 0.0;
        else if ((d0 > 0.0) != (d1 > 0.0) && fabs(s) > fabs(3.0 * d0)) s = 3.0 * d0;
        m[idx] = s;
    }
    free(h);
    free(d);
}

/* Pressure and dp/de of the tabulated EoS at e.  Below the first node:
 * p = p0 e / e0; above the last: linear with the end slope. */
static void table_eval(const ora_params* P, double e, double* p, double* dpde)
{
    const int n = P->ntab;
    const double* x = P->etab;
    const double* y = P->ptab;
    const double* m = P->mtab;
    if (e <= x[0]) {
        *p = y[0] * e / x[0];
        *dpde = y[0] / x[0];
        return;
    }
    if (e >= x[n - 1]) {
        *p = y[n - 1] + m[n - 1] * (e - x[n - 1]);
        *dpde = m[n - 1];
        return;
    }
    /* interval [x[lo], x[lo+1]) containing e, by bisection */
    int lo = 0, hi = n - 1;
    while (hi - lo > 1) {
        int mid = (lo + hi) / 2;
        if (x[mid] <= e) lo = mid; else hi = mid;
    }
    double h = x[lo + 1] - x[lo];
    double t = (e - x[lo]) / h;
    double t2 = t * t, t3 = t2 * t;
    double h00 = 2.0 * t3 - 3.0 * t2 + 1.0;
    double h10 = t3 - 2.0 * t2 + t;
    double h01 = -2.0 * t3 + 3.0 * t2;
    double h11 = t3 - t2;
    *p = h00 * y[lo] + h10 * h * m[lo] + h01 * y[lo + 1] + h11 * h * m[lo + 1];
    double d00 = (6.0 * t2 - 6.0 * t) / h;
    double d10 = 3.0 * t2 - 4.0 * t + 1.0;
    double d01 = (-6.0 * t2 + 6.0 * t) / h;
    double d11 = 3.0 * t2 - 2.0 * t;
    *dpde = d00 * y[lo] + d10 * m[lo] + d01 * y[lo + 1] + d11 * m[lo + 1];
}

void ora_eos_eval(const ora_params* P, int64_t n, const double* e, double* p, double* dpde)
{
    for (int64_t i = 0; i < n; i++) {
        if (P->eos == EOS_IDEAL) { p[i] = P->cs2 * e[i]; dpde[i] = P->cs2; }
        else table_eval(P, e[i], &p[i], &dpde[i]);
    }
}

/* ---------------------------------------------------------------------- */
/* Conserved -> primitive (Sec. 2.6)                                       */
/* ---------------------------------------------------------------------- */

/* Recover (e, p, v) from U = (E, Mx, My, Mz).  The paper writes the inverse
 * of the prim->cons relations as the fixed point v = |M| / (E + p(E - |M| v))
 * with e = E - M.v.  For p = c e this is the quadratic
 *   c |M| v^2 - (1 + c) E v + |M| = 0,
 * whose root below one is v = 2|M| / ((1+c)E + sqrt((1+c)^2 E^2 - 4 c |M|^2));
 * the velocity vector is v M/|M| = 2 M / ((1+c)E + sqrt(...)).
 * For a tabulated p(e) the same fixed point is the root of
 *   g(e) = e - E + |M|^2 / (E + p(e))
 * on [E (1 - m^2), E], m = |M|/E, found here by bisection.
 * With the charge R (Sec. 2.6, eq. for v): n = R sqrt(1 - v^2).  For p = c e
 * or the table, p does not depend on n and v is found as above.  For the
 * ideal gas p(e, n) = (gamma - 1) max(e - n, 0) the fixed point
 *   v = |M| / (E + p(E - |M| v, R sqrt(1 - v^2)))
 * is solved by bisection in v on [0, |M|/E] (p >= 0 puts the root there; it
 * is unique because p -> v = |M| / (E + p) maps the roots one to one onto
 * those of the decreasing function (gamma - 1)(e(p) - n(p)) - p).  For
 * gamma = 1 (pressureless dust) p = 0 and v = |M|/E directly.
 * Returns the (possibly clamped) momentum used, through Mu[3];
 * prim = (e, p, vx, vy, vz, n).  Returns 0 for a state counted as bad
 * (E <= 0, a non-finite component, or R < 0 with the ideal gas), which is
 * evaluated as the zero state, else 1. */
static int con2prim(const ora_params* P, const double* U, double prim[6], double Mu[3],
                     ora_counters* cnt)
{
    double E = U[0];
    double Mx = U[1], My = U[2], Mz = U[3];
    double R = P->charge ? U[4] : 0.0;
    cnt->n_calls++;
    if (!(E > 0.0) || !isfinite(E) || !isfinite(Mx) || !isfinite(My) || !isfinite(Mz) || !isfinite(R) ||
        (P->eos == EOS_GAMMA && !(R >= 0.0))) {
        cnt->n_bad++;
        for (int q = 0; q < 6; q++) prim[q] = 0.0;
        Mu[0] = 0.0; Mu[1] = 0.0; Mu[2] = 0.0;
        return 0;
    }
    double M2 = Mx * Mx + My * My + Mz * Mz;
    double Mlim = ORA_MMAX * E;
    if (M2 > Mlim * Mlim) {
        double s = Mlim / sqrt(M2);
        Mx = Mx * s; My = My * s; Mz = Mz * s;
        M2 = Mx * Mx + My * My + Mz * Mz;
        cnt->n_floor++;
    }
    Mu[0] = Mx; Mu[1] = My; Mu[2] = Mz;
    double e, p, vx, vy, vz;
    if (P->eos == EOS_IDEAL) {
        double c = P->cs2;
        double q = 1.0 + c;
        double s = sqrt(q * q * E * E - 4.0 * c * M2);
        double den = q * E + s;
        vx = 2.0 * Mx / den;
        vy = 2.0 * My / den;
        vz = 2.0 * Mz / den;
        e = E - (Mx * vx + My * vy + Mz * vz);
        p = c * e;
    } else if (P->eos == EOS_TABLE) {
        double lo = E - M2 / E; /* E (1 - m^2) */
        double hi = E;
        double pe, dp;
        int it = 0;
        if (M2 == 0.0) { lo = E; hi = E; }
        while (hi - lo > 1e-15 * hi && it < 200) {
            double mid = 0.5 * (lo + hi);
            table_eval(P, mid, &pe, &dp);
            double g = mid - E + M2 / (E + pe);
            if (g > 0.0) hi = mid; else lo = mid;
            it++;
        }
        cnt->n_iter += it;
        e = 0.5 * (lo + hi);
        table_eval(P, e, &p, &dp);
        double w = E + p;
        vx = Mx / w;
        vy = My / w;
        vz = Mz / w;
    } else {
        const double gm1 = P->gamma - 1.0;
        const double M = sqrt(M2);
        double v = 0.0;
        if (gm1 == 0.0) {
            v = M / E;  /* pressureless dust: the fixed point is explicit */
        } else if (M2 > 0.0) {
            double lo = 0.0, hi = M / E;
            int it = 0;
            while (it < 200) {  /* to the last bit: stop when the midpoint is an end */
                double mid = 0.5 * (lo + hi);
                if (!(mid > lo && mid < hi)) break;
                double pm = gm1 * fmax(E - M * mid - R * sqrt(1.0 - mid * mid), 0.0);
                if (mid - M / (E + pm) > 0.0) hi = mid; else lo = mid;
                it++;
            }
            cnt->n_iter += it;
            v = 0.5 * (lo + hi);
        }
        e = E - M * v;
        p = gm1 * fmax(e - R * sqrt(1.0 - v * v), 0.0);
        double w = E + p;
        vx = Mx / w;
        vy = My / w;
        vz = Mz / w;
    }
    prim[0] = e; prim[1] = p; prim[2] = vx; prim[3] = vy; prim[4] = vz;
    prim[5] = R * sqrt(1.0 - (vx * vx + vy * vy + vz * vz));
    return 1;
}

/* R and n may be NULL (no charge). */
void ora_con2prim(const ora_params* P, int64_t n, const double* E, const double* Mx,
                  const double* My, const double* Mz, const double* R, double* e, double* p,
                  double* vx, double* vy, double* vz, double* nrest, ora_counters* cnt)
{
    ora_counters c = {0, 0, 0, 0};
    for (int64_t i = 0; i < n; i++) {
        double U[NCMAX] = {E[i], Mx[i], My[i], Mz[i], R ? R[i] : 0.0}, pr[6], Mu[3];
        con2prim(P, U, pr, Mu, &c);
        e[i] = pr[0]; p[i] = pr[1]; vx[i] = pr[2]; vy[i] = pr[3]; vz[i] = pr[4];
        if (nrest) nrest[i] = pr[5];
    }
    if (cnt) *cnt = c;
}

/* ---------------------------------------------------------------------- */
/* Physical flux along axis d (Sec. 2.1, flux vectors F, G, H)             */
/* ---------------------------------------------------------------------- */

static void flux(const ora_params* P, int d, const double* U, double* F, ora_counters* cnt)
{
    double pr[6], Mu[3];
    const int ncp = ncomp(P);
    if (!con2prim(P, U, pr, Mu, cnt)) {  /* the zero state: zero flux */
        for (int q = 0; q < ncp; q++) F[q] = 0.0;
        return;
    }
    double p = pr[1];
    double vd = pr[2 + d];
    F[0] = (U[0] + p) * vd;
    F[1] = Mu[0] * vd;
    F[2] = Mu[1] * vd;
    F[3] = Mu[2] * vd;
    F[1 + d] = F[1 + d] + p;
    if (P->charge) F[4] = U[4] * vd;
}

void ora_flux(const ora_params* P, int32_t d, int64_t n, const double* U /* (nc, n) */,
              double* F /* (nc, n) */)
{
    ora_counters c = {0, 0, 0, 0};
    const int ncp = ncomp(P);
    for (int64_t i = 0; i < n; i++) {
        double u[NCMAX], f[NCMAX];
        for (int q = 0; q < ncp; q++) u[q] = U[q * n + i];
        flux(P, d, u, f, &c);
        for (int q = 0; q < ncp; q++) F[q * n + i] = f[q];
    }
}

/* ---------------------------------------------------------------------- */
/* Slope limiters (Sec. 2.5) in two-argument form                          */
/* ---------------------------------------------------------------------- */

/* phi(a, b) = xi(r) a with a = U_i - U_{i-1}, b = U_{i+1} - U_i, r = b / a.
 * "Same sign" means both non-zero with equal signs (no product is formed). */
static int same_sign(double a, double b)
{
    return (a > 0.0 && b > 0.0) || (a < 0.0 && b < 0.0);
}

static double limiter(int lim, double a, double b)
{
    switch (lim) {
    case LIM_NONE: /* central slope 1/2 (U_{i+1} - U_{i-1}) */
        return 0.5 * (a + b);
    case LIM_MINMOD: /* xi = max(0, min(1, r)) */
        if (!same_sign(a, b)) return 0.0;
        return copysign(fmin(fabs(a), fabs(b)), a);
    case LIM_SUPERBEE: /* xi = max(0, min(2r, 1), min(r, 2)) */
        if (!same_sign(a, b)) return 0.0;
        return copysign(fmax(fmin(2.0 * fabs(b), fabs(a)), fmin(fabs(b), 2.0 * fabs(a))), a);
    case LIM_MC: /* xi = max(0, min(2r, (1+r)/2, 2)) */
        if (!same_sign(a, b)) return 0.0;
        return copysign(fmin(fmin(2.0 * fabs(a), 2.0 * fabs(b)), 0.5 * fabs(a + b)), a);
    case LIM_VANLEER: /* xi = (r + |r|) / (1 + |r|) */
        if (!same_sign(a, b)) return 0.0;
        return 2.0 * a * b / (a + b);
    case LIM_VANALBADA: /* xi = (r^2 + r) / (r^2 + 1), not clipped */
        /* slopes so small that a^2 + b^2 is zero in double (|a|, |b| < 1e-154) give 0 */
        if (a * a + b * b == 0.0) return 0.0;
        return a * b * (a + b) / (a * a + b * b);
    default:
        return 0.0;
    }
}

void ora_limiter(int32_t lim, int64_t n, const double* a, const double* b, double* out)
{
    for (int64_t i = 0; i < n; i++) out[i] = limiter(lim, a[i], b[i]);
}

/* ---------------------------------------------------------------------- */
/* MUSTA-FORCE interface flux (Sec. 2.4)                                   */
/* ---------------------------------------------------------------------- */

/* k stages of: centred FORCE flux from (U_L, U_R); if more stages follow,
 * the local predictor update of U_L and U_R.  lam = dt / dx_d. */
static void musta(const ora_params* P, int d, double lam, const double* UL0,
                  const double* UR0, double* Fh, ora_counters* cnt)
{
    double UL[NCMAX], UR[NCMAX], FL[NCMAX], FR[NCMAX], Us[NCMAX], Flw[NCMAX], Flf[NCMAX];
    const double alpha = P->alpha;
    const double lp = P->predictor_alpha ? alpha * lam : lam;  /* predictor coefficient */
    const int ncp = ncomp(P);
    for (int c = 0; c < ncp; c++) { UL[c] = UL0[c]; UR[c] = UR0[c]; }
    for (int l = 1; l <= P->k; l++) {
        flux(P, d, UL, FL, cnt);
        flux(P, d, UR, FR, cnt);
        /* Lax-Wendroff (Richtmyer) flux */
        for (int c = 0; c < ncp; c++)
            Us[c] = 0.5 * (UL[c] + UR[c]) - 0.5 * alpha * lam * (FR[c] - FL[c]);
        flux(P, d, Us, Flw, cnt);
        /* Lax-Friedrichs flux */
        for (int c = 0; c < ncp; c++)
            Flf[c] = 0.5 * (FL[c] + FR[c]) - (UR[c] - UL[c]) / (2.0 * alpha * lam);
        /* FORCE = mean of the two */
        for (int c = 0; c < ncp; c++) Fh[c] = 0.5 * (Flw[c] + Flf[c]);
        if (l < P->k) {
            for (int c = 0; c < ncp; c++) {
                UL[c] = UL[c] - lp * (Fh[c] - FL[c]);
                UR[c] = UR[c] - lp * (FR[c] - Fh[c]);
            }
        }
    }
}

void ora_musta(const ora_params* P, int32_t d, double lam, int64_t n, const double* UL,
               const double* UR, double* F)
{
    ora_counters c = {0, 0, 0, 0};
    const int ncp = ncomp(P);
    for (int64_t i = 0; i < n; i++) {
        double l[NCMAX], r[NCMAX], f[NCMAX];
        for (int q = 0; q < ncp; q++) { l[q] = UL[q * n + i]; r[q] = UR[q * n + i]; }
        musta(P, d, lam, l, r, f, &c);
        for (int q = 0; q < ncp; q++) F[q * n + i] = f[q];
    }
}

/* ---------------------------------------------------------------------- */
/* One line: reconstruction, Hancock half step, interface fluxes, -dF/dx   */
/* ---------------------------------------------------------------------- */

/* u: N+4 padded cells (u[j] is cell j-2).  Adds -(F_{i+1/2} - F_{i-1/2})/dx
 * into out[i], i = 0..N-1.  dl: Hancock corrections of cells -1..N (dl[j] is
 * cell j-1) from the unsplit step, or NULL for the per-axis step. */
static void line_rhs(const ora_params* P, int d, int N, double lam, double dxd,
                     double (*u)[NCMAX], double (*uLt)[NCMAX], double (*uRt)[NCMAX], double (*F)[NCMAX],
                     double (*out)[NCMAX], const double (*dl)[NCMAX], ora_counters* cnt)
{
    const int ncp = ncomp(P);
    /* MUSCL reconstruction and Hancock half step for cells -1..N */
    for (int i = -1; i <= N; i++) {
        const double* um = u[i + 1];
        const double* u0 = u[i + 2];
        const double* up = u[i + 3];
        double UL[NCMAX], UR[NCMAX], FLc[NCMAX], FRc[NCMAX];
        for (int c = 0; c < ncp; c++) {
            double a = u0[c] - um[c];
            double b = up[c] - u0[c];
            double D = limiter(P->limiter, a, b);
            UL[c] = u0[c] - 0.5 * D;
            UR[c] = u0[c] + 0.5 * D;
        }
        if (dl) {
            for (int c = 0; c < ncp; c++) {
                uLt[i + 1][c] = UL[c] + dl[i + 1][c];
                uRt[i + 1][c] = UR[c] + dl[i + 1][c];
            }
            continue;
        }
        flux(P, d, UL, FLc, cnt);
        flux(P, d, UR, FRc, cnt);
        for (int c = 0; c < ncp; c++) {
            double delta = 0.5 * lam * (FLc[c] - FRc[c]);
            uLt[i + 1][c] = UL[c] + delta;
            uRt[i + 1][c] = UR[c] + delta;
        }
    }
    /* interface fluxes F_{i+1/2}, i = -1..N-1, from (Ut^R_i, Ut^L_{i+1}) */
    for (int i = -1; i <= N - 1; i++) musta(P, d, lam, uRt[i + 1], uLt[i + 2], F[i + 1], cnt);
    for (int i = 0; i < N; i++)
        for (int c = 0; c < ncp; c++) out[i][c] = -(F[i + 1][c] - F[i][c]) / dxd;
}

static int64_t ghost_index(int j, int N, int bc)
{
    if (j >= 0 && j < N) return j;
    if (bc == BC_PERIODIC) return ((j % N) + N) % N;
    return j < 0 ? 0 : N - 1;
}

/* Unsplit Hancock corrections on the grid extended by one ghost cell per
 * side, (nx+2)(ny+2)(nz+2) cells, cell (i,j,k) at ((k+1)(ny+2) + j+1)(nx+2) + i+1:
 *   delta = sum_d (dt / (2 dx_d)) (F_d(U^{L,d}) - F_d(U^{R,d})),
 * with U^{L,d}, U^{R,d} = U -/+ phi_d / 2 the limited faces along each axis,
 * and the state outside the grid from the boundary conditions per axis. */
static double* unsplit_corrections(const ora_params* P, const double* U, double dt, ora_counters* cnt_out)
{
    const int nx = P->n[0], ny = P->n[1], nz = P->n[2];
    const int64_t ncell = (int64_t)nx * ny * nz;
    const int ex = nx + 2, ey = ny + 2, ez = nz + 2;
    const int64_t next = (int64_t)ex * ey * ez;
    const int ncp = ncomp(P);
    double* dl = malloc(sizeof(double) * NCMAX * (size_t)next);
    int64_t nf = 0, nb = 0, ni = 0, nc = 0;
#pragma omp parallel for schedule(static) reduction(+ : nf, nb, ni, nc)
    for (int64_t e = 0; e < next; e++) {
        const int i = (int)(e % ex) - 1, j = (int)((e / ex) % ey) - 1, k = (int)(e / ((int64_t)ex * ey)) - 1;
        ora_counters cnt = {0, 0, 0, 0};
        double delta[NCMAX] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int d = 0; d < 3; d++) {
            double w[3][NCMAX];  /* cells -1, 0, +1 along d */
            for (int s = -1; s <= 1; s++) {
                int q[3] = {i, j, k};
                q[d] += s;
                const int64_t idx = ghost_index(q[0], nx, P->bc[0]) +
                                    nx * (ghost_index(q[1], ny, P->bc[1]) + ny * ghost_index(q[2], nz, P->bc[2]));
                for (int c = 0; c < ncp; c++) w[s + 1][c] = U[c * ncell + idx];
            }
            double UL[NCMAX], UR[NCMAX], FL[NCMAX], FR[NCMAX];
            for (int c = 0; c < ncp; c++) {
                const double D = limiter(P->limiter, w[1][c] - w[0][c], w[2][c] - w[1][c]);
                UL[c] = w[1][c] - 0.5 * D;
                UR[c] = w[1][c] + 0.5 * D;
            }
            flux(P, d, UL, FL, &cnt);
            flux(P, d, UR, FR, &cnt);
            const double lam = dt / P->dx[d];
            for (int c = 0; c < ncp; c++) delta[c] = delta[c] + 0.5 * lam * (FL[c] - FR[c]);
        }
        for (int c = 0; c < ncp; c++) dl[NCMAX * e + c] = delta[c];
        nf += cnt.n_floor; nb += cnt.n_bad; ni += cnt.n_iter; nc += cnt.n_calls;
    }
    cnt_out->n_floor += nf; cnt_out->n_bad += nb; cnt_out->n_iter += ni; cnt_out->n_calls += nc;
    return dl;
}

/* L(U, t) = -(dF/dx + dG/dy + dH/dz) + S, summed as ((Lx + Ly) + Lz) + S. */
static void rhs(const ora_params* P, const double* U, double t, double dt, double* L,
                ora_counters* cnt_out)
{
    const int nx = P->n[0], ny = P->n[1], nz = P->n[2];
    const int64_t ncell = (int64_t)nx * ny * nz;
    const int64_t stride[3] = {1, nx, (int64_t)nx * ny};
    const int ncp = ncomp(P);
    memset(L, 0, sizeof(double) * (size_t)ncomp(P) * (size_t)ncell);
    int64_t nf = 0, nb = 0, ni = 0, nc = 0;
    ora_counters cpre = {0, 0, 0, 0};
    double* dl3 = P->unsplit_hancock ? unsplit_corrections(P, U, dt, &cpre) : NULL;
    const int64_t estride[3] = {1, nx + 2, (int64_t)(nx + 2) * (ny + 2)};
    for (int d = 0; d < 3; d++) {
        const int N = P->n[d];
        const double lam = dt / P->dx[d];
        const int a1 = (d == 0) ? 1 : 0;           /* the two other axes */
        const int a2 = (d == 2) ? 1 : 2;
        const int64_t nlines = ncell / N;
#pragma omp parallel reduction(+ : nf, nb, ni, nc)
        {
            double(*u)[NCMAX] = malloc(sizeof(double[NCMAX]) * (size_t)(N + 4));
            double(*uLt)[NCMAX] = malloc(sizeof(double[NCMAX]) * (size_t)(N + 2));
            double(*uRt)[NCMAX] = malloc(sizeof(double[NCMAX]) * (size_t)(N + 2));
            double(*F)[NCMAX] = malloc(sizeof(double[NCMAX]) * (size_t)(N + 1));
            double(*out)[NCMAX] = malloc(sizeof(double[NCMAX]) * (size_t)N);
            double(*dl)[NCMAX] = dl3 ? malloc(sizeof(double[NCMAX]) * (size_t)(N + 2)) : NULL;
            ora_counters cnt = {0, 0, 0, 0};
#pragma omp for schedule(static)
            for (int64_t line = 0; line < nlines; line++) {
                int64_t i1 = line % P->n[a1];
                int64_t i2 = line / P->n[a1];
                int64_t base = i1 * stride[a1] + i2 * stride[a2];
                for (int j = -2; j < N + 2; j++) {
                    int64_t idx = base + ghost_index(j, N, P->bc[d]) * stride[d];
                    for (int c = 0; c < ncp; c++) u[j + 2][c] = U[c * ncell + idx];
                }
                if (dl) {  /* corrections of cells -1..N along the line */
                    const int64_t ebase = (i1 + 1) * estride[a1] + (i2 + 1) * estride[a2];
                    for (int j = -1; j <= N; j++)
                        for (int c = 0; c < ncp; c++) dl[j + 1][c] = dl3[NCMAX * (ebase + (int64_t)(j + 1) * estride[d]) + c];
                }
                line_rhs(P, d, N, lam, P->dx[d], u, uLt, uRt, F, out, (const double(*)[NCMAX])dl, &cnt);
                for (int j = 0; j < N; j++) {
                    int64_t idx = base + (int64_t)j * stride[d];
                    for (int c = 0; c < ncp; c++) L[c * ncell + idx] = L[c * ncell + idx] + out[j][c];
                }
            }
            nf += cnt.n_floor; nb += cnt.n_bad; ni += cnt.n_iter; nc += cnt.n_calls;
            free(u); free(uLt); free(uRt); free(F); free(out); free(dl);
        }
    }
    if (P->jet) {
        /* S = v dE/dx G_sigma(x - x_jet(t)) (1, v, 0, 0), sampled at cell centres */
        const double s2 = P->jet_sigma * P->jet_sigma;
        const double norm = pow(2.0 * M_PI * s2, -1.5);
        const double xj = P->jet_x0[0] + P->jet_v * t;
        const double yj = P->jet_x0[1], zj = P->jet_x0[2];
#pragma omp parallel for schedule(static)
        for (int64_t idx = 0; idx < ncell; idx++) {
            int64_t i = idx % nx, j = (idx / nx) % ny, kk = idx / ((int64_t)nx * ny);
            double x = P->xlo[0] + (i + 0.5) * P->dx[0] - xj;
            double y = P->xlo[1] + (j + 0.5) * P->dx[1] - yj;
            double z = P->xlo[2] + (kk + 0.5) * P->dx[2] - zj;
            double G = norm * exp(-(x * x + y * y + z * z) / (2.0 * s2));
            double SE = P->jet_v * P->jet_dedx * G;
            L[idx] = L[idx] + SE;
            L[ncell + idx] = L[ncell + idx] + P->jet_v * SE;
        }
    }
    free(dl3);
    nf += cpre.n_floor; nb += cpre.n_bad; ni += cpre.n_iter; nc += cpre.n_calls;
    cnt_out->n_floor += nf; cnt_out->n_bad += nb; cnt_out->n_iter += ni; cnt_out->n_calls += nc;
}

void ora_rhs(const ora_params* P, const double* U, double t, double dt, double* L,
             ora_counters* cnt)
{
    ora_counters c = {0, 0, 0, 0};
    rhs(P, U, t, dt, L, &c);
    if (cnt) *cnt = c;
}

/* ---------------------------------------------------------------------- */
/* Diagnostics                                                             */
/* ---------------------------------------------------------------------- */

/* Largest |characteristic speed| over cells and axes:
 * lambda_pm = [v_d (1 - cs^2) +- cs sqrt((1 - v^2)(1 - v_d^2 - (v^2 - v_d^2) cs^2))] / (1 - v^2 cs^2),
 * with cs^2 = dp/de at the cell's e. */
double ora_max_speed(const ora_params* P, const double* U, ora_counters* cnt_out)
{
    const int64_t ncell = (int64_t)P->n[0] * P->n[1] * P->n[2];
    const int ncp = ncomp(P);
    double smax = 0.0;
    int64_t nf = 0, nb = 0, ni = 0, nc = 0;
#pragma omp parallel reduction(max : smax) reduction(+ : nf, nb, ni, nc)
    {
        ora_counters cnt = {0, 0, 0, 0};
#pragma omp for schedule(static)
        for (int64_t i = 0; i < ncell; i++) {
            double u[NCMAX], pr[6], Mu[3], p, c2;
            for (int q = 0; q < ncp; q++) u[q] = U[q * ncell + i];
            con2prim(P, u, pr, Mu, &cnt);
            if (P->eos == EOS_IDEAL) c2 = P->cs2;
            else if (P->eos == EOS_TABLE) table_eval(P, pr[0], &p, &c2);
            else c2 = pr[1] > 0.0 ? P->gamma * pr[1] / (pr[0] + pr[1]) : 0.0;  /* ideal gas */
            double cs = sqrt(c2);
            double v2 = pr[2] * pr[2] + pr[3] * pr[3] + pr[4] * pr[4];
            for (int d = 0; d < 3; d++) {
                double vd = pr[2 + d];
                double rad = (1.0 - v2) * (1.0 - vd * vd - (v2 - vd * vd) * c2);
                double root = cs * sqrt(rad > 0.0 ? rad : 0.0);
                double den = 1.0 - v2 * c2;
                double lp = (vd * (1.0 - c2) + root) / den;
                double lm = (vd * (1.0 - c2) - root) / den;
                double s = fmax(fabs(lp), fabs(lm));
                if (s > smax) smax = s;
            }
        }
        nf += cnt.n_floor; nb += cnt.n_bad; ni += cnt.n_iter; nc += cnt.n_calls;
    }
    if (cnt_out) {
        cnt_out->n_floor += nf; cnt_out->n_bad += nb; cnt_out->n_iter += ni; cnt_out->n_calls += nc;
    }
    return smax;
}

/* Neumaier-compensated sums of each conserved component times the cell volume. */
void ora_totals(const ora_params* P, const double* U, double* out /* ncomp */)
{
    const int64_t ncell = (int64_t)P->n[0] * P->n[1] * P->n[2];
    const double dV = P->dx[0] * P->dx[1] * P->dx[2];
    for (int c = 0; c < ncomp(P); c++) {
        double s = 0.0, comp = 0.0;
        for (int64_t i = 0; i < ncell; i++) {
            double x = U[c * ncell + i];
            double t = s + x;
            if (fabs(s) >= fabs(x)) comp += (s - t) + x;
            else comp += (x - t) + s;
            s = t;
        }
        out[c] = (s + comp) * dV;
    }
}

/* ---------------------------------------------------------------------- */
/* Runge-Kutta steps (Sec. 2.3)                                            */
/* ---------------------------------------------------------------------- */

typedef struct {
    double smax;      /* max characteristic speed over the end-of-step states */
    ora_counters cnt; /* summed over all L evaluations of the call */
} ora_stats;

/* Advance U (ncomp x ncell, SoA, x fastest) by nsteps steps of size dt from t0. */
int ora_step(const ora_params* P, double* U, double t0, double dt, int32_t nsteps,
             ora_stats* st)
{
    const int64_t ncell = (int64_t)P->n[0] * P->n[1] * P->n[2];
    const int64_t nv = ncomp(P) * ncell;
    double* L = malloc(sizeof(double) * (size_t)nv);
    double* U1 = malloc(sizeof(double) * (size_t)nv);
    double* U2 = (P->rk == 3) ? malloc(sizeof(double) * (size_t)nv) : NULL;
    if (!L || !U1 || (P->rk == 3 && !U2)) { free(L); free(U1); free(U2); return -1; }
    ora_counters cnt = {0, 0, 0, 0};
    double smax = 0.0;
    double t = t0;
    for (int s = 0; s < nsteps; s++) {
        /* U1 = U + dt L(U) */
        rhs(P, U, t, dt, L, &cnt);
#pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < nv; i++) U1[i] = U[i] + dt * L[i];
        if (P->rk == 3) {
            /* U2 = 3/4 U + 1/4 U1 + 1/4 dt L(U1) */
            rhs(P, U1, t + dt, dt, L, &cnt);
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < nv; i++) U2[i] = 0.75 * U[i] + 0.25 * U1[i] + 0.25 * (dt * L[i]);
            /* U^{n+1} = 1/3 U + 2/3 U2 + 2/3 dt L(U2) */
            rhs(P, U2, t + 0.5 * dt, dt, L, &cnt);
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < nv; i++)
                U[i] = (1.0 / 3.0) * U[i] + (2.0 / 3.0) * U2[i] + (2.0 / 3.0) * (dt * L[i]);
        } else {
            /* U^{n+1} = 1/2 (U + U1 + dt L(U1)) */
            rhs(P, U1, t + dt, dt, L, &cnt);
#pragma omp parallel for schedule(static)
            for (int64_t i = 0; i < nv; i++) U[i] = 0.5 * (U[i] + U1[i] + dt * L[i]);
        }
        t = t0 + (s + 1) * dt;
        ora_counters dummy = {0, 0, 0, 0};
        double sm = ora_max_speed(P, U, &dummy);
        if (sm > smax) smax = sm;
    }
    free(L); free(U1); free(U2);
    if (st) { st->smax = smax; st->cnt = cnt; }
    return 0;
}

int ora_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void ora_set_num_threads(int32_t n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
