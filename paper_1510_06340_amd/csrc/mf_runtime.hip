// mf_runtime.hip -- host runtime and C ABI (include/mf.h) of the MUSTA-FORCE
// library: handles, library-owned scratch, the per-step launch sequence of
// the dimensionally split Runge-Kutta stages, statistics and reductions.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "../../include/mf.h"
#include "mf_kernels.hpp"
#include "mf_mlp.hpp"

using namespace mf;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg)
{
    g_err = msg;
    return code;
}

#define MF_HIP(call)                                                                           \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) return fail(MF_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

constexpr int kTotalsBlocks = 512;

struct Event {
    mf_grid_desc d;
    int64_t ncell = 0;
    int nc = 4;                        // conserved components: 4, or 5 with the charge R
    void* U[kMaxComp] = {};            // caller-owned
    void* U1[kMaxComp] = {};           // RK stage 1 output
    void* U2[kMaxComp] = {};           // RK3 stage 2 output
    void* L[kMaxComp] = {};            // flux-divergence accumulator
    void* DL = nullptr;  // MF_FLAG_UNSPLIT_HANCOCK: 4 (n0+2)(n1+2)(n2+2) corrections
    int64_t dl_n = 0;    // (n0+2)(n1+2)(n2+2)
    double t = 0.0;
    int64_t steps = 0;
    bool jet = false;
    double jet_x0[3] = {0, 0, 0};
    double jet_v = 0, jet_dedx = 0, jet_sigma = 1;
};

size_t elem_size(int dtype) { return dtype == MF_F32 ? 4 : 8; }

}  // namespace

struct mf_grid_s {
    std::vector<Event> ev;
    hipStream_t stream = nullptr;
    int eos_kind = -1;
    double cs2 = 1.0 / 3.0;
    EosTable table{};               // device view of the tabulated EoS
    double gamma = 5.0 / 3.0;       // MF_EOS_GAMMA: adiabatic index
    void* table_dev = nullptr;      // its records (library-owned)
    float* seed_params = nullptr;   // seed network parameters (device, MF_MLP_PARAMS)
    float* seed_grid = nullptr;     // its predictions on the (ln E, |M|/E) grid
    SeedNorm seed_norm{};
    bool has_seed = false;
    int seg_override[3] = {0, 0, 0};
    int block = 256;
    unsigned long long* dstats = nullptr;  // (n_events + 1) * ST_WORDS; the last slot is scratch
    double* dpartial = nullptr;            // kTotalsBlocks * kMaxComp
    double* dtot = nullptr;                // n_events * kMaxComp
    std::vector<void*> allocs;
    // kernel timing (mf_set_profiling)
    bool profiling = false;
    struct Timed {
        int axis;
        hipEvent_t start, stop;
    };
    std::vector<Timed> timed;       // launches recorded since the last read
    std::vector<hipEvent_t> pool;   // recycled events

    // batched stepping (mf_batch_step): tuned shapes, device tables, captured step
    struct Batch {
        bool tuned = false;
        int shape[3] = {0, 0, 0};   // x: chunks per wavefront; y, z: cells per thread
        int block[3] = {256, 256, 256};
        std::vector<double> dt;     // the dt set the tables and the graph were built for
        void* tab = nullptr;        // SweepArgs[nstage][3][ne]
        int64_t* tiles = nullptr;   // [3][ne + 1] tile prefix per axis
        int64_t total[3] = {0, 0, 0};
        unsigned int* counters = nullptr;  // one per (stage, axis)
        double* t_dev = nullptr;    // event times
        double* dt_dev = nullptr;
        std::vector<double> t_host; // staging for the time upload
        hipStream_t stream = nullptr;
        hipEvent_t ev_in = nullptr, ev_out = nullptr;
        hipGraphExec_t exec = nullptr;
        hipGraph_t graph = nullptr;
    } batch;

    ~mf_grid_s()
    {
        if (batch.exec) (void)hipGraphExecDestroy(batch.exec);
        if (batch.graph) (void)hipGraphDestroy(batch.graph);
        if (batch.ev_in) (void)hipEventDestroy(batch.ev_in);
        if (batch.ev_out) (void)hipEventDestroy(batch.ev_out);
        if (batch.stream) (void)hipStreamDestroy(batch.stream);
        for (auto& t : timed) {
            (void)hipEventDestroy(t.start);
            (void)hipEventDestroy(t.stop);
        }
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        for (void* p : allocs) (void)hipFree(p);
    }
    hipError_t take_event(hipEvent_t* e)
    {
        if (!pool.empty()) {
            *e = pool.back();
            pool.pop_back();
            return hipSuccess;
        }
        return hipEventCreate(e);
    }
    void release(void* p)
    {
        if (!p) return;
        (void)hipFree(p);
        allocs.erase(std::remove(allocs.begin(), allocs.end(), p), allocs.end());
    }
    int alloc(void** p, size_t bytes)
    {
        *p = nullptr;
        if (bytes == 0) bytes = 8;
        hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess) {
            *p = nullptr;
            (void)hipGetLastError();
            return fail(MF_ERR_NOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed: " +
                                          hipGetErrorString(e));
        }
        allocs.push_back(*p);
        return MF_OK;
    }
};

namespace {

// Sweep geometry of axis d on an (nx, ny, nz) grid with x fastest.
struct AxisGeom {
    int N, n_fast, axis_f, axis_s;
    int64_t nlines, stride_d, stride_f, stride_s;
};

AxisGeom axis_geom(const int32_t n[3], int d)
{
    const int64_t nx = n[0], ny = n[1], nz = n[2];
    AxisGeom g;
    if (d == 0) {
        g = {n[0], n[1], 1, 2, ny * nz, 1, nx, nx * ny};
    } else if (d == 1) {
        g = {n[1], n[0], 0, 2, nx * nz, nx, 1, nx * ny};
    } else {
        g = {n[2], n[0], 0, 1, nx * ny, nx * ny, 1, nx};
    }
    return g;
}

// x sweep (lanes along x): chunks of 64 row items per wavefront, chosen to
// give about two full rounds of the kernel's resident wavefronts on every
// SIMD (waves_per_simd, from its occupancy).  Where con2prim runs a Newton
// solve (the table EoS, the ideal gas) the cost per cell varies with the local
// iterations, and smaller work units (about four rounds) balance it better.
int auto_chunks_x(const AxisGeom& g, bool newton, int waves_per_simd)
{
    const int64_t items = g.nlines * ((int64_t)g.N + 2);
    const int64_t target_waves = 256LL * 4 * waves_per_simd * (newton ? 4 : 2);
    int64_t cpw = (items + 64 * target_waves - 1) / (64 * target_waves);
    return (int)std::max<int64_t>(1, std::min<int64_t>(cpw, 64));
}

// Cells per thread along the sweep axis: enough segments for two full rounds
// of the kernel's resident wavefronts (waves_per_simd, from its occupancy) on
// every SIMD of the 256 compute units (the second round balances the tail),
// but at least 16 cells per segment (each segment recomputes two
// reconstructions and one interface).  Where con2prim runs a Newton solve
// (uneven, latency-bound cost per cell): 16 wavefronts per SIMD (five rounds
// of three) and at least 8 cells.
int auto_seg(const AxisGeom& g, bool newton, int waves_per_simd)
{
    const int64_t target_threads = 256LL * 4 * 64 * (newton ? 16 : 2 * waves_per_simd);
    int64_t min_cells = newton ? 8 : 16;
    // Small grids (under one wavefront per compute unit at that length) take
    // segments down to 4 cells: the march's latency, not the overlap, bounds them.
    if (g.nlines * ((g.N + min_cells - 1) / min_cells) < 256LL * 64) min_cells = 4;
    int64_t nseg = (target_threads + g.nlines - 1) / g.nlines;
    nseg = std::max<int64_t>(1, std::min<int64_t>(nseg, (g.N + min_cells - 1) / min_cells));
    return (int)((g.N + nseg - 1) / nseg);
}

template <typename T>
void set_axis_const(AxisConst<T>& ac, double dt, double dx, double alpha, bool predictor_alpha)
{
    const double lam = dt / dx;
    ac.lam = (T)(predictor_alpha ? alpha * lam : lam);
    ac.half_lam = (T)(0.5 * lam);
    ac.half_alam = (T)(0.5 * alpha * lam);
    ac.inv_2alam = (T)(1.0 / (2.0 * alpha * lam));
    ac.inv_2dx = (T)(0.5 / dx);
}

// Argument block of one axis sweep d of one Runge-Kutta stage of event ev.
// seg: cells per thread (y, z) or chunks of 64 row items per wavefront (x).
template <typename T>
SweepArgs<T> make_sweep_args(const Event& ev, int d, int seg, unsigned long long* stats, void* const uin[],
                             void* const u0[], void* const out[], int kind, double dt, bool want_smax)
{
    const AxisGeom geo = axis_geom(ev.d.n, d);
    SweepArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    for (int c = 0; c < ev.nc; c++) {
        a.u[c] = (const T*)uin[c];
        a.L[c] = (T*)ev.L[c];
        a.u0[c] = (const T*)u0[c];
        a.out[c] = (T*)out[c];
    }
    a.nlines = geo.nlines;
    a.stride_d = geo.stride_d;
    a.stride_f = geo.stride_f;
    a.stride_s = geo.stride_s;
    a.N = geo.N;
    a.n_fast = geo.n_fast;
    a.seg = seg;
    a.periodic = ev.d.bc[d] == MF_BC_PERIODIC;
    a.k = ev.d.musta_k;
    a.kind = kind;
    a.want_smax = want_smax ? 1 : 0;
    a.axis_f = geo.axis_f;
    a.axis_s = geo.axis_s;
    set_axis_const(a.ac, dt, ev.d.dx[d], ev.d.alpha, (ev.d.flags & MF_FLAG_PREDICTOR_ALPHA) != 0);
    a.dt = (T)dt;
    if (ev.DL) {
        const int64_t es[3] = {1, (int64_t)ev.d.n[0] + 2, ((int64_t)ev.d.n[0] + 2) * ((int64_t)ev.d.n[1] + 2)};
        a.dl = (const T*)ev.DL;
        a.dl_n = ev.dl_n;
        a.estride_d = es[d];
        a.estride_f = es[geo.axis_f];
        a.estride_s = es[geo.axis_s];
    }
    if (ev.jet && d == 2) {
        a.jet_pos[0] = ev.jet_x0[0];
        a.jet_pos[1] = ev.jet_x0[1];
        a.jet_pos[2] = ev.jet_x0[2];
        a.jet_ve = ev.jet_v * ev.jet_dedx;
        a.jet_v = ev.jet_v;
        a.jet_norm = std::pow(2.0 * M_PI * ev.jet_sigma * ev.jet_sigma, -1.5);
        a.jet_inv2s2 = 1.0 / (2.0 * ev.jet_sigma * ev.jet_sigma);
    }
    for (int q = 0; q < 3; q++) {
        a.origin[q] = ev.d.origin[q];
        a.dx[q] = ev.d.dx[q];
    }
    a.stats = stats;
    return a;
}

// Tiles (blocks of the per-event kernels) of axis d at the given shape.
int64_t axis_tiles(const Event& ev, int d, int seg, int block)
{
    const AxisGeom geo = axis_geom(ev.d.n, d);
    if (d == 0) {
        const int64_t items = geo.nlines * ((int64_t)geo.N + 2);
        const int64_t waves = (items + 64LL * seg - 1) / (64LL * seg);
        return (waves * 64 + block - 1) / block;
    }
    const int64_t nseg = (geo.N + seg - 1) / seg;
    return ((geo.nlines + block - 1) / block) * nseg;
}

int default_shape(const Event& ev, int d, bool newton, int waves_per_simd)
{
    const AxisGeom geo = axis_geom(ev.d.n, d);
    return d == 0 ? auto_chunks_x(geo, newton, waves_per_simd) : auto_seg(geo, newton, waves_per_simd);
}

// What a stage needs besides the event: the stream, launch-shape overrides
// (0 = automatic), the block size, whether con2prim runs a Newton solve (the
// table EoS and the ideal gas: finer work units) and whether the EoS is
// tabulated, and the handle that collects kernel timings (nullptr: no timing).
struct StageCtx {
    hipStream_t stream;
    int seg_override[3];
    int block;
    bool newton;
    bool table;
    mf_grid_s* prof;
};

StageCtx stage_ctx(mf_grid_s* g)
{
    StageCtx c;
    c.stream = g->stream;
    for (int q = 0; q < 3; q++) c.seg_override[q] = g->seg_override[q];
    c.block = g->block;
    c.newton = g->eos_kind == MF_EOS_TABLE || g->eos_kind == MF_EOS_GAMMA;
    c.table = g->eos_kind == MF_EOS_TABLE;
    c.prof = g->profiling ? g : nullptr;
    return c;
}

// Sweeps with the charge exist for FP64 with p = c e (a passive charge) and the ideal gas.
template <typename T, class Eos>
constexpr bool kChargeSweeps = std::is_same<T, double>::value &&
                               (std::is_same<Eos, EosIdeal<double>>::value || std::is_same<Eos, EosGamma>::value);

template <typename T, class Eos>
int run_stage(const StageCtx& cx, const Eos& eos, Event& ev, unsigned long long* stats, void* const uin[],
              void* const u0[], void* const out[], int kind, double dt, double ts, bool want_smax)
{
    if constexpr (!kChargeSweeps<T, Eos>) {
        if (ev.nc == 5) return fail(MF_ERR_ARG, "the charge runs in FP64 with p = c e or the ideal gas");
    }
    if constexpr (std::is_same<Eos, EosGamma>::value) {
        if (ev.nc != 5) return fail(MF_ERR_ARG, "the ideal gas needs the charge");
    }
    if constexpr (std::is_same<Eos, EosGamma>::value) {
        if (ev.DL) return fail(MF_ERR_ARG, "the unsplit Hancock ablation carries no charge");
    } else if (ev.DL) {  // unsplit Hancock ablation: the three-axis corrections of the stage input
        UnsplitArgs<T> ua;
        std::memset(&ua, 0, sizeof(ua));
        for (int c = 0; c < 4; c++) ua.u[c] = (const T*)uin[c];
        ua.dl = (T*)ev.DL;
        ua.dl_n = ev.dl_n;
        for (int q = 0; q < 3; q++) {
            ua.n[q] = ev.d.n[q];
            ua.periodic[q] = ev.d.bc[q] == MF_BC_PERIODIC;
            ua.half_lam[q] = (T)(0.5 * (dt / ev.d.dx[q]));
        }
        ua.stats = stats;
        hipError_t e = launch_unsplit_delta<T, Eos>(ev.d.limiter, cx.stream, ua, eos);
        if (e != hipSuccess) return fail(MF_ERR_HIP, std::string("unsplit launch: ") + hipGetErrorString(e));
    }
    for (int d = 0; d < 3; d++) {
        const AxisGeom geo = axis_geom(ev.d.n, d);
        int waves = 0;
        if (cx.seg_override[d] <= 0) {
            if constexpr (kChargeSweeps<T, Eos>) {
                if (ev.nc == 5) waves = sweep_waves_per_simd_charge<Eos>(d, ev.d.limiter, cx.block);
            }
            if constexpr (!std::is_same<Eos, EosGamma>::value) {
                if (ev.nc == 4) waves = sweep_waves_per_simd<T, Eos>(d, ev.d.limiter, ev.jet && d == 2, cx.block);
            }
        }
        // the ideal gas's x sweep (four wavefronts per SIMD) ran 5% slower with the finer chunks
        const bool fine = cx.newton && (d > 0 || cx.table);
        int seg = cx.seg_override[d] > 0 ? cx.seg_override[d] : default_shape(ev, d, fine, waves);
        if (d > 0) seg = std::min(seg, geo.N);
        SweepArgs<T> a = make_sweep_args<T>(ev, d, seg, stats, uin, u0, out, kind, dt, want_smax);
        const bool jet = ev.jet && d == 2;
        if (jet) a.jet_pos[0] = ev.jet_x0[0] + ev.jet_v * ts;
        dim3 block(cx.block);
        dim3 grid;
        if (d == 0) {
            grid = dim3((unsigned)axis_tiles(ev, 0, a.seg, cx.block), 1);
        } else {
            const int64_t nseg = (geo.N + a.seg - 1) / a.seg;
            grid = dim3((unsigned)((geo.nlines + cx.block - 1) / cx.block), (unsigned)nseg);
        }
        mf_grid_s::Timed tm{d, nullptr, nullptr};
        if (cx.prof) {
            MF_HIP(cx.prof->take_event(&tm.start));
            MF_HIP(cx.prof->take_event(&tm.stop));
            MF_HIP(hipEventRecord(tm.start, cx.stream));
        }
        hipError_t e = hipErrorInvalidValue;
        if constexpr (kChargeSweeps<T, Eos>) {
            if (ev.nc == 5) e = launch_sweep_charge<Eos>(d, ev.d.limiter, grid, block, cx.stream, a, eos);
        }
        if constexpr (!std::is_same<Eos, EosGamma>::value) {
            if (ev.nc == 4)
                e = ev.DL ? launch_sweep_unsplit<T, Eos>(d, ev.d.limiter, jet, grid, block, cx.stream, a, eos)
                          : launch_sweep<T, Eos>(d, ev.d.limiter, jet, grid, block, cx.stream, a, eos);
        }
        if (e != hipSuccess) return fail(MF_ERR_HIP, std::string("sweep launch: ") + hipGetErrorString(e));
        if (cx.prof) {
            MF_HIP(hipEventRecord(tm.stop, cx.stream));
            cx.prof->timed.push_back(tm);
        }
    }
    return MF_OK;
}

template <typename T, class Eos>
int run_steps_eos(const StageCtx& g, const Eos& eos, Event& ev, unsigned long long* stats, double dt, int nsteps)
{
    int rc;
    for (int s = 0; s < nsteps; s++) {
        const double t = ev.t;
        if (ev.d.rk_order == 3) {
            if ((rc = run_stage<T>(g, eos, ev, stats, ev.U, ev.U, ev.U1, RK_FIRST, dt, t, false))) return rc;
            if ((rc = run_stage<T>(g, eos, ev, stats, ev.U1, ev.U, ev.U2, RK3_MID, dt, t + dt, false))) return rc;
            if ((rc = run_stage<T>(g, eos, ev, stats, ev.U2, ev.U, ev.U, RK3_LAST, dt, t + 0.5 * dt, true)))
                return rc;
        } else {
            if ((rc = run_stage<T>(g, eos, ev, stats, ev.U, ev.U, ev.U1, RK_FIRST, dt, t, false))) return rc;
            if ((rc = run_stage<T>(g, eos, ev, stats, ev.U1, ev.U, ev.U, RK2_LAST, dt, t + dt, true))) return rc;
        }
        ev.steps++;
        ev.t = ev.t + dt;
    }
    return MF_OK;
}

int run_steps(mf_grid_s* g, Event& ev, unsigned long long* stats, double dt, int nsteps)
{
    const StageCtx cx = stage_ctx(g);
    if (g->eos_kind == MF_EOS_TABLE) return run_steps_eos<double>(cx, g->table, ev, stats, dt, nsteps);
    if (g->eos_kind == MF_EOS_GAMMA) return run_steps_eos<double>(cx, EosGamma::make(g->gamma), ev, stats, dt, nsteps);
    if (ev.d.dtype == MF_F32) return run_steps_eos<float>(cx, EosIdeal<float>::make(g->cs2), ev, stats, dt, nsteps);
    return run_steps_eos<double>(cx, EosIdeal<double>::make(g->cs2), ev, stats, dt, nsteps);
}

// Monotone piecewise-cubic node slopes (Fritsch & Carlson 1980), interior
// slopes the weighted harmonic mean of Fritsch & Butland (1984), end slopes
// from the one-sided three-point formula with the monotonicity clamp.
void monotone_slopes(int n, const double* x, const double* y, std::vector<double>& m)
{
    m.assign(n, 0.0);
    std::vector<double> h(n - 1), del(n - 1);
    for (int i = 0; i + 1 < n; i++) {
        h[i] = x[i + 1] - x[i];
        del[i] = (y[i + 1] - y[i]) / h[i];
    }
    if (n == 2) {
        m[0] = m[1] = del[0];
        return;
    }
    for (int i = 1; i + 1 < n; i++) {
        const bool same = (del[i - 1] > 0.0 && del[i] > 0.0) || (del[i - 1] < 0.0 && del[i] < 0.0);
        if (!same) continue;
        const double w1 = 2.0 * h[i] + h[i - 1];
        const double w2 = h[i] + 2.0 * h[i - 1];
        m[i] = (w1 + w2) / (w1 / del[i - 1] + w2 / del[i]);
    }
    auto end_slope = [](double h0, double h1, double d0, double d1) {
        double sl = ((2.0 * h0 + h1) * d0 - h0 * d1) / (h0 + h1);
        if (sl == 0.0 || d0 == 0.0 || (sl > 0.0) != (d0 > 0.0)) return 0.0;
        if ((d0 > 0.0) != (d1 > 0.0) && std::fabs(sl) > std::fabs(3.0 * d0)) return 3.0 * d0;
        return sl;
    };
    m[0] = end_slope(h[0], h[1], del[0], del[1]);
    m[n - 1] = end_slope(h[n - 2], h[n - 3], del[n - 2], del[n - 3]);
}

// Conservation sums of one event's nc components into out[nc] (device); partial: kMaxComp
// kTotalsBlocks doubles (device).
template <typename T>
int enqueue_totals(hipStream_t stream, double* partial, const Event& ev, double* out)
{
    TotalsArgs<T> a;
    std::memset(&a, 0, sizeof(a));
    for (int c = 0; c < ev.nc; c++) a.U[c] = (const T*)ev.U[c];
    a.n = ev.ncell;
    a.partial = partial;
    const double dV = ev.d.dx[0] * ev.d.dx[1] * ev.d.dx[2];
    hipError_t e = launch_totals<T>(stream, a, ev.nc, kTotalsBlocks, dV, out);
    if (e != hipSuccess) return fail(MF_ERR_HIP, std::string("totals launch: ") + hipGetErrorString(e));
    return MF_OK;
}

int enqueue_totals_any(hipStream_t stream, double* partial, const Event& ev, double* out)
{
    return ev.d.dtype == MF_F32 ? enqueue_totals<float>(stream, partial, ev, out)
                                : enqueue_totals<double>(stream, partial, ev, out);
}

// Host statistics of one event from its device counters w[ST_WORDS] and totals tot[0..3].
void fill_stats(const Event& ev, const unsigned long long* w, const double* tot, double dt, mf_stats& s)
{
    std::memset(&s, 0, sizeof(s));
    double smax;
    std::memcpy(&smax, &w[ST_SMAX], sizeof(double));
    s.t = ev.t;
    s.steps = ev.steps;
    s.smax = smax;
    const double dxmin = std::min(ev.d.dx[0], std::min(ev.d.dx[1], ev.d.dx[2]));
    s.courant = smax * dt / dxmin;
    for (int c = 0; c < 4; c++) s.totals[c] = tot[c];
    s.n_floor = (int64_t)w[ST_FLOOR];
    s.n_bad = (int64_t)w[ST_BAD];
    s.newton_iters = (int64_t)w[ST_ITERS];
    s.n_fallback = (int64_t)w[ST_FALLBACK];
}

// MF_FLAG_STRICT verdict of one event's statistics.
int strict_status(const mf_grid_desc& d, const mf_stats& st, int event)
{
    if (!(d.flags & MF_FLAG_STRICT)) return MF_OK;
    if (st.n_bad > 0 || st.n_floor > 0)
        return fail(MF_ERR_UNPHYSICAL, "event " + std::to_string(event) + ": unphysical states met (" +
                                           std::to_string(st.n_bad) + " bad, " + std::to_string(st.n_floor) +
                                           " clamped)");
    if (d.alpha * st.courant > 1.0)
        return fail(MF_ERR_CFL, "event " + std::to_string(event) + ": alpha * Courant number exceeds 1");
    return MF_OK;
}


// ---------------------------------------------------------------------------
// Batched stepping: all events advance together, one persistent launch per
// axis sweep and Runge-Kutta stage over a tile queue, the whole step captured
// once into a HIP graph and replayed.
// ---------------------------------------------------------------------------
struct StageIO {
    void* const* uin;
    void* const* u0;
    void* const* out;
    int kind;
    double t_off_frac;  // stage time = t + t_off_frac * dt
    bool want_smax;
};

int stage_io(const Event& ev, int stage, StageIO& io)
{
    if (ev.d.rk_order == 3) {
        if (stage == 0) io = {ev.U, ev.U, ev.U1, RK_FIRST, 0.0, false};
        else if (stage == 1) io = {ev.U1, ev.U, ev.U2, RK3_MID, 1.0, false};
        else io = {ev.U2, ev.U, ev.U, RK3_LAST, 0.5, true};
    } else {
        if (stage == 0) io = {ev.U, ev.U, ev.U1, RK_FIRST, 0.0, false};
        else io = {ev.U1, ev.U, ev.U, RK2_LAST, 1.0, true};
    }
    return MF_OK;
}

// Host image of the batch tables for the given stages/axes and shapes.
template <typename T>
void build_tables(mf_grid_s* g, const double* dt, int nstage, const int shape[3], const int block[3],
                  std::vector<SweepArgs<T>>& tab, std::vector<int64_t>& tiles, int64_t total[3])
{
    const int ne = (int)g->ev.size();
    auto& b = g->batch;
    tab.assign((size_t)nstage * 3 * ne, SweepArgs<T>());
    tiles.assign((size_t)3 * (ne + 1), 0);
    for (int d = 0; d < 3; d++) {
        int64_t acc = 0;
        for (int e = 0; e < ne; e++) {
            const Event& ev = g->ev[e];
            int seg = shape[d];
            if (d > 0) seg = std::min(seg, ev.d.n[d]);
            tiles[(size_t)d * (ne + 1) + e] = acc;
            acc += axis_tiles(ev, d, seg, block[d]);
            for (int st = 0; st < nstage; st++) {
                StageIO io;
                stage_io(ev, st, io);
                SweepArgs<T> a = make_sweep_args<T>(ev, d, seg, g->dstats + (size_t)ST_WORDS * e, io.uin, io.u0,
                                                    io.out, io.kind, dt[e], io.want_smax);
                a.t_ptr = b.t_dev + e;
                a.t_off = io.t_off_frac * dt[e];
                tab[((size_t)st * 3 + d) * ne + e] = a;
            }
        }
        tiles[(size_t)d * (ne + 1) + ne] = acc;
        total[d] = acc;
    }
}

int ensure_batch_buffers(mf_grid_s* g)
{
    auto& b = g->batch;
    const int ne = (int)g->ev.size();
    int rc = MF_OK;
    if (!b.stream) MF_HIP(hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking));
    if (!b.ev_in) MF_HIP(hipEventCreateWithFlags(&b.ev_in, hipEventDisableTiming));
    if (!b.ev_out) MF_HIP(hipEventCreateWithFlags(&b.ev_out, hipEventDisableTiming));
    if (!b.tab) rc = g->alloc(&b.tab, sizeof(SweepArgs<double>) * 3 * 3 * (size_t)ne);
    if (!rc && !b.tiles) rc = g->alloc((void**)&b.tiles, sizeof(int64_t) * 3 * (size_t)(ne + 1));
    if (!rc && !b.counters) rc = g->alloc((void**)&b.counters, sizeof(unsigned int) * 16);
    if (!rc && !b.t_dev) rc = g->alloc((void**)&b.t_dev, sizeof(double) * (size_t)ne);
    if (!rc && !b.dt_dev) rc = g->alloc((void**)&b.dt_dev, sizeof(double) * (size_t)ne);
    return rc;
}

// Autotuner: for each axis, time the stage-1 sweep (which writes only
// library-owned buffers: L and the stage state U1) over all events at every
// candidate (block size, shape) and keep the fastest.
template <typename T, class Eos>
int batch_tune(mf_grid_s* g, const Eos& eos, const double* dt)
{
    auto& b = g->batch;
    const int ne = (int)g->ev.size();
    bool jet = false;
    for (const Event& ev : g->ev) jet = jet || ev.jet;
    const int lim = g->ev[0].d.limiter;
    hipEvent_t t0, t1;
    MF_HIP(hipEventCreate(&t0));
    MF_HIP(hipEventCreate(&t1));
    std::vector<double> tnow(ne);
    for (int e = 0; e < ne; e++) tnow[e] = g->ev[e].t;
    MF_HIP(hipMemcpyAsync(b.t_dev, tnow.data(), sizeof(double) * ne, hipMemcpyHostToDevice, b.stream));
    const int cand_x[4] = {4, 8, 16, 32};
    const int cand_yz[5] = {8, 16, 32, 64, 128};
    const int blocks[2] = {128, 256};
    int best_shape[3] = {0, 0, 0}, best_block[3] = {256, 256, 256};
    for (int d = 0; d < 3; d++) {
        float best = 1e30f;
        for (int bi = 0; bi < 2; bi++) {
            const int ncand = d == 0 ? 4 : 5;
            for (int ci = 0; ci < ncand; ci++) {
                int shape[3] = {8, 64, 64}, block[3] = {256, 256, 256};
                for (int q = 0; q < 3; q++) {
                    shape[q] = best_shape[q] ? best_shape[q] : shape[q];
                    block[q] = best_block[q];
                }
                shape[d] = d == 0 ? cand_x[ci] : cand_yz[ci];
                block[d] = blocks[bi];
                std::vector<SweepArgs<T>> tab;
                std::vector<int64_t> tiles;
                int64_t total[3];
                build_tables<T>(g, dt, 1, shape, block, tab, tiles, total);
                MF_HIP(hipMemcpyAsync(b.tab, tab.data(), sizeof(SweepArgs<T>) * tab.size(), hipMemcpyHostToDevice,
                                      b.stream));
                MF_HIP(hipMemcpyAsync(b.tiles, tiles.data(), sizeof(int64_t) * tiles.size(), hipMemcpyHostToDevice,
                                      b.stream));
                float ms = 0.0f;
                for (int rep = 0; rep < 2; rep++) {
                    hipError_t e = launch_fill_u32(b.stream, b.counters, 1, 0u);
                    if (e != hipSuccess) return fail(MF_ERR_HIP, hipGetErrorString(e));
                    MF_HIP(hipEventRecord(t0, b.stream));
                    e = launch_batch_sweep<T, Eos>(d, lim, jet, (const SweepArgs<T>*)b.tab + (size_t)d * ne,
                                                   b.tiles + (size_t)d * (ne + 1), ne, b.counters, total[d],
                                                   block[d], b.stream, eos);
                    if (e != hipSuccess) return fail(MF_ERR_HIP, std::string("tuning launch: ") + hipGetErrorString(e));
                    MF_HIP(hipEventRecord(t1, b.stream));
                    MF_HIP(hipEventSynchronize(t1));
                    MF_HIP(hipEventElapsedTime(&ms, t0, t1));
                }
                if (ms < best) {
                    best = ms;
                    best_shape[d] = shape[d];
                    best_block[d] = block[d];
                }
            }
        }
    }
    (void)hipEventDestroy(t0);
    (void)hipEventDestroy(t1);
    for (int q = 0; q < 3; q++) {
        b.shape[q] = best_shape[q];
        b.block[q] = best_block[q];
    }
    b.tuned = true;
    return MF_OK;
}

template <typename T, class Eos>
int batch_build(mf_grid_s* g, const Eos& eos, const double* dt)
{
    auto& b = g->batch;
    const int ne = (int)g->ev.size();
    const int nstage = g->ev[0].d.rk_order == 3 ? 3 : 2;
    bool jet = false;
    for (const Event& ev : g->ev) jet = jet || ev.jet;
    const int lim = g->ev[0].d.limiter;
    std::vector<SweepArgs<T>> tab;
    std::vector<int64_t> tiles;
    build_tables<T>(g, dt, nstage, b.shape, b.block, tab, tiles, b.total);
    MF_HIP(hipMemcpyAsync(b.tab, tab.data(), sizeof(SweepArgs<T>) * tab.size(), hipMemcpyHostToDevice, b.stream));
    MF_HIP(hipMemcpyAsync(b.tiles, tiles.data(), sizeof(int64_t) * tiles.size(), hipMemcpyHostToDevice, b.stream));
    MF_HIP(hipMemcpyAsync(b.dt_dev, dt, sizeof(double) * ne, hipMemcpyHostToDevice, b.stream));
    MF_HIP(hipStreamSynchronize(b.stream));
    if (b.exec) {
        (void)hipGraphExecDestroy(b.exec);
        b.exec = nullptr;
    }
    if (b.graph) {
        (void)hipGraphDestroy(b.graph);
        b.graph = nullptr;
    }
    MF_HIP(hipStreamBeginCapture(b.stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = launch_fill_u32(b.stream, b.counters, nstage * 3, 0u);
    for (int st = 0; st < nstage && e == hipSuccess; st++) {
        for (int d = 0; d < 3 && e == hipSuccess; d++) {
            e = launch_batch_sweep<T, Eos>(d, lim, jet, (const SweepArgs<T>*)b.tab + ((size_t)st * 3 + d) * ne,
                                           b.tiles + (size_t)d * (ne + 1), ne, b.counters + st * 3 + d, b.total[d],
                                           b.block[d], b.stream, eos);
        }
    }
    if (e == hipSuccess) e = launch_advance_time(b.stream, b.t_dev, b.dt_dev, ne);
    hipGraph_t graph = nullptr;
    hipError_t ec = hipStreamEndCapture(b.stream, &graph);
    if (e != hipSuccess) return fail(MF_ERR_HIP, std::string("batched step capture: ") + hipGetErrorString(e));
    if (ec != hipSuccess) return fail(MF_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
    b.graph = graph;
    MF_HIP(hipGraphInstantiate(&b.exec, b.graph, nullptr, nullptr, 0));
    b.dt.assign(dt, dt + ne);
    return MF_OK;
}

template <typename T, class Eos>
int batch_prepare(mf_grid_s* g, const Eos& eos, const double* dt)
{
    auto& b = g->batch;
    const int ne = (int)g->ev.size();
    int rc;
    if (!b.tuned) {
        if (g->seg_override[0] > 0 && g->seg_override[1] > 0 && g->seg_override[2] > 0) {
            for (int q = 0; q < 3; q++) {
                b.shape[q] = g->seg_override[q];
                b.block[q] = g->block;
            }
            b.tuned = true;
        } else if ((rc = batch_tune<T>(g, eos, dt))) {
            return rc;
        }
    }
    const bool same = b.exec && (int)b.dt.size() == ne && std::equal(b.dt.begin(), b.dt.end(), dt);
    if (!same && (rc = batch_build<T>(g, eos, dt))) return rc;
    return MF_OK;
}

int batch_prepare_any(mf_grid_s* g, const double* dt)
{
    if (g->eos_kind == MF_EOS_TABLE) return batch_prepare<double>(g, g->table, dt);
    if (g->ev[0].d.dtype == MF_F32) return batch_prepare<float>(g, EosIdeal<float>::make(g->cs2), dt);
    return batch_prepare<double>(g, EosIdeal<double>::make(g->cs2), dt);
}

// Upload the seed network and fill its prediction grid over
// ln E in [ln 1e-4, ln 1e4] (kSeedG0 points) and |M|/E in [0, 1] (kSeedG1 points).

int install_seed(mf_grid_s* g, const mf_surrogate& s)
{
    const int H = MF_MLP_HIDDEN;
    std::vector<float> P(MF_MLP_PARAMS);
    size_t o = 0;
    for (int i = 0; i < 2 * H; i++) P[o++] = s.w1[i];
    for (int i = 0; i < H; i++) P[o++] = s.b1[i];
    for (int i = 0; i < H * H; i++) P[o++] = s.w2[i];
    for (int i = 0; i < H; i++) P[o++] = s.b2[i];
    for (int i = 0; i < H; i++) P[o++] = s.w3[i];
    P[o++] = s.b3;
    SeedNorm nrm;
    for (int q = 0; q < 2; q++) {
        nrm.in_shift[q] = s.in_shift[q];
        nrm.in_scale[q] = s.in_scale[q];
    }
    nrm.out_shift = s.out_shift;
    nrm.out_scale = s.out_scale;
    nrm.output = s.output;
    int rc = g->alloc((void**)&g->seed_params, sizeof(float) * MF_MLP_PARAMS);
    if (!rc) rc = g->alloc((void**)&g->seed_grid, sizeof(float) * kSeedG0 * kSeedG1);
    if (rc) return rc;
    float* X = nullptr;
    rc = g->alloc((void**)&X, sizeof(float) * 2 * kSeedG0 * kSeedG1);
    if (rc) return rc;
    std::vector<float> hx((size_t)2 * kSeedG0 * kSeedG1), hy((size_t)kSeedG0 * kSeedG1);
    const double dl = (kSeedLnHi - kSeedLnLo) / (kSeedG0 - 1);
    for (int i = 0; i < kSeedG0; i++)
        for (int j = 0; j < kSeedG1; j++) {
            const size_t k = (size_t)i * kSeedG1 + j;
            hx[2 * k] = (float)((kSeedLnLo + i * dl - nrm.in_shift[0]) * nrm.in_scale[0]);
            hx[2 * k + 1] = (float)(((double)j / (kSeedG1 - 1) - nrm.in_shift[1]) * nrm.in_scale[1]);
        }
    MF_HIP(hipMemcpy(g->seed_params, P.data(), sizeof(float) * P.size(), hipMemcpyHostToDevice));
    MF_HIP(hipMemcpy(X, hx.data(), sizeof(float) * hx.size(), hipMemcpyHostToDevice));
    hipError_t e = mlp_forward(g->seed_params, X, (int64_t)kSeedG0 * kSeedG1, g->seed_grid, nullptr);
    if (e != hipSuccess) return fail(MF_ERR_HIP, std::string("seed grid: ") + hipGetErrorString(e));
    MF_HIP(hipDeviceSynchronize());
    MF_HIP(hipMemcpy(hy.data(), g->seed_grid, sizeof(float) * hy.size(), hipMemcpyDeviceToHost));
    for (float& v : hy) v = v * nrm.out_scale + nrm.out_shift;  // ln e or the bracket fraction
    MF_HIP(hipMemcpy(g->seed_grid, hy.data(), sizeof(float) * hy.size(), hipMemcpyHostToDevice));
    g->release(X);
    g->seed_norm = nrm;
    g->has_seed = true;
    EosTable& t = g->table;
    t.seed = g->seed_grid;
    t.seed_output = nrm.output;
    return MF_OK;
}

int check_desc(const mf_grid_desc& d)
{
    for (int q = 0; q < 3; q++) {
        if (d.n[q] < 1) return fail(MF_ERR_ARG, "grid size n[" + std::to_string(q) + "] must be >= 1");
        if (!(d.dx[q] > 0.0) || !std::isfinite(d.dx[q])) return fail(MF_ERR_ARG, "dx must be finite and > 0");
        if (d.bc[q] != MF_BC_OUTFLOW && d.bc[q] != MF_BC_PERIODIC) return fail(MF_ERR_ARG, "unknown boundary code");
        if (!std::isfinite(d.origin[q])) return fail(MF_ERR_ARG, "origin must be finite");
    }
    if ((int64_t)d.n[0] * d.n[1] > INT32_MAX || (int64_t)d.n[0] * d.n[1] * d.n[2] > (int64_t)1 << 40)
        return fail(MF_ERR_ARG, "grid too large");
    if (d.dtype != MF_F64 && d.dtype != MF_F32) return fail(MF_ERR_ARG, "unknown dtype");
    if (d.limiter < MF_LIM_NONE || d.limiter > MF_LIM_VANALBADA) return fail(MF_ERR_ARG, "unknown limiter");
    if (d.musta_k < 1 || d.musta_k > 64) return fail(MF_ERR_ARG, "musta_k must be in [1, 64]");
    if (d.rk_order != 2 && d.rk_order != 3) return fail(MF_ERR_ARG, "rk_order must be 2 or 3");
    if (!(d.alpha > 0.0) || !std::isfinite(d.alpha)) return fail(MF_ERR_ARG, "alpha must be finite and > 0");
    if (d.flags & ~(MF_FLAG_STRICT | MF_FLAG_PREDICTOR_ALPHA | MF_FLAG_UNSPLIT_HANCOCK | MF_FLAG_CHARGE))
        return fail(MF_ERR_ARG, "unknown flag bits");
    if ((d.flags & MF_FLAG_CHARGE) && d.dtype != MF_F64) return fail(MF_ERR_ARG, "the charge runs in FP64 only");
    if ((d.flags & MF_FLAG_CHARGE) && (d.flags & MF_FLAG_UNSPLIT_HANCOCK))
        return fail(MF_ERR_ARG, "the unsplit Hancock ablation carries no charge");
    return MF_OK;
}

}  // namespace

// Partial gradients of mf_mlp_grad_noalloc: one row of MF_MLP_PARAMS + 1 floats per
// block (64 samples) of the gradient kernel, for up to MF_MLP_NOALLOC_MAX_N samples
// (1.1 MB).  Every device holds its own copy; host code reaches it only through the
// address that hipGetSymbolAddress returns on that device (the name itself is a
// host stand-in).
static constexpr int64_t kNoallocFloats = ((int64_t)(MF_MLP_NOALLOC_MAX_N + 63) / 64) * (MF_MLP_PARAMS + 1);
static __device__ __align__(256) float scratch[kNoallocFloats];

namespace {

constexpr int kMaxDevices = 64;

// Device address of `scratch` on the current device, looked up once per device.
int noalloc_scratch(float** out)
{
    static std::mutex mu;
    static float* ptr[kMaxDevices] = {};
    int dev = 0;
    MF_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(MF_ERR_ARG, "device index beyond the library's table");
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[dev]) {
        void* p = nullptr;
        MF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return fail(MF_ERR_HIP, "hipGetSymbolAddress returned no address for the scratch array");
        ptr[dev] = (float*)p;
    }
    *out = ptr[dev];
    return MF_OK;
}

}  // namespace

extern "C" {

const char* mf_last_error(void) { return g_err.c_str(); }

int mf_grid_init(mf_grid_t* out, const mf_grid_desc* descs, int32_t n_events, void* const* U_dev, void* stream)
{
    g_err.clear();
    if (!out || !descs || !U_dev) return fail(MF_ERR_ARG, "null argument");
    *out = nullptr;
    if (n_events < 1) return fail(MF_ERR_ARG, "n_events must be >= 1");
    const bool charge = (descs[0].flags & MF_FLAG_CHARGE) != 0;
    const int nc = charge ? 5 : 4;
    for (int i = 0; i < n_events; i++) {
        int rc = check_desc(descs[i]);
        if (rc) return rc;
        if (((descs[i].flags & MF_FLAG_CHARGE) != 0) != charge)
            return fail(MF_ERR_ARG, "all events of a handle carry the charge or none does");
        for (int c = 0; c < nc; c++)
            if (!U_dev[(int64_t)nc * i + c]) return fail(MF_ERR_ARG, "null state pointer");
    }
    mf_grid_s* g = new (std::nothrow) mf_grid_s();
    if (!g) return fail(MF_ERR_NOMEM, "host allocation failed");
    g->stream = (hipStream_t)stream;
    g->ev.resize(n_events);
    int rc = MF_OK;
    for (int i = 0; i < n_events && rc == MF_OK; i++) {
        Event& ev = g->ev[i];
        ev.d = descs[i];
        ev.nc = nc;
        ev.ncell = (int64_t)ev.d.n[0] * ev.d.n[1] * ev.d.n[2];
        const size_t bytes = (size_t)ev.ncell * elem_size(ev.d.dtype);
        for (int c = 0; c < nc && rc == MF_OK; c++) {
            ev.U[c] = U_dev[(int64_t)nc * i + c];
            rc = g->alloc(&ev.U1[c], bytes);
            if (rc == MF_OK) rc = g->alloc(&ev.L[c], bytes);
            if (rc == MF_OK && ev.d.rk_order == 3) rc = g->alloc(&ev.U2[c], bytes);
        }
        if (rc == MF_OK && (ev.d.flags & MF_FLAG_UNSPLIT_HANCOCK)) {
            ev.dl_n = ((int64_t)ev.d.n[0] + 2) * ((int64_t)ev.d.n[1] + 2) * ((int64_t)ev.d.n[2] + 2);
            rc = g->alloc(&ev.DL, (size_t)ev.dl_n * 4 * elem_size(ev.d.dtype));
        }
    }
    if (rc == MF_OK) rc = g->alloc((void**)&g->dstats, sizeof(unsigned long long) * ST_WORDS * (n_events + 1));
    if (rc == MF_OK) rc = g->alloc((void**)&g->dpartial, sizeof(double) * kMaxComp * kTotalsBlocks);
    if (rc == MF_OK) rc = g->alloc((void**)&g->dtot, sizeof(double) * kMaxComp * n_events);
    if (rc != MF_OK) {
        std::string msg = g_err;
        delete g;
        return fail(rc, msg);
    }
    *out = g;
    return MF_OK;
}

int mf_grid_free(mf_grid_t g)
{
    if (!g) return fail(MF_ERR_ARG, "null handle");
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    else (void)hipDeviceSynchronize();
    delete g;
    return MF_OK;
}

int mf_set_eos(mf_grid_t g, int32_t kind, double cs2, const double* e_tab, const double* p_tab, int32_t n_tab,
               const mf_surrogate* s)
{
    if (!g) return fail(MF_ERR_ARG, "null handle");
    const bool charge = g->ev[0].nc == 5;
    if (kind == MF_EOS_IDEAL) {
        if (!(cs2 > 0.0 && cs2 < 1.0)) return fail(MF_ERR_ARG, "cs2 must be in (0, 1)");
        if (s) return fail(MF_ERR_ARG, "a surrogate needs the table EoS");
        g->eos_kind = MF_EOS_IDEAL;
        g->cs2 = cs2;
        return MF_OK;
    }
    if (kind == MF_EOS_GAMMA) {  // cs2 carries the adiabatic index
        if (!(cs2 >= 1.0 && cs2 <= 2.0)) return fail(MF_ERR_ARG, "the adiabatic index must be in [1, 2]");
        if (!charge) return fail(MF_ERR_ARG, "the ideal gas needs the charge (MF_FLAG_CHARGE)");
        if (s) return fail(MF_ERR_ARG, "a surrogate needs the table EoS");
        g->eos_kind = MF_EOS_GAMMA;
        g->gamma = cs2;
        return MF_OK;
    }
    if (kind != MF_EOS_TABLE) return fail(MF_ERR_ARG, "unknown EoS kind");
    if (charge) return fail(MF_ERR_ARG, "the tabulated EoS carries no charge");
    if (!e_tab || !p_tab || n_tab < 3) return fail(MF_ERR_ARG, "table EoS needs n_tab >= 3 host nodes");
    for (const Event& ev : g->ev)
        if (ev.d.dtype != MF_F64) return fail(MF_ERR_ARG, "the table EoS runs in FP64 only");
    for (int i = 0; i < n_tab; i++) {
        if (!(e_tab[i] > 0.0) || !std::isfinite(e_tab[i]) || !(p_tab[i] >= 0.0) || !std::isfinite(p_tab[i]) ||
            !(p_tab[i] < e_tab[i]))
            return fail(MF_ERR_ARG, "table nodes need e > 0 and 0 <= p < e");
        if (i > 0 && (!(e_tab[i] > e_tab[i - 1]) || p_tab[i] < p_tab[i - 1]))
            return fail(MF_ERR_ARG, "table e must increase strictly and p must not decrease");
    }
    if (s && (s->hidden != MF_MLP_HIDDEN || !s->w1 || !s->b1 || !s->w2 || !s->b2 || !s->w3 ||
              (s->output != 0 && s->output != 1)))
        return fail(MF_ERR_ARG, "the seed network must be 2-64-64-1 with all weights and output 0 or 1");
    std::vector<double> m;
    monotone_slopes(n_tab, e_tab, p_tab, m);
    // n + 1 pieces (x, w, y, c1, c2, c3): p = y + t (c1 + t (c2 + t c3)), t = (e - x) w, the
    // piece holding e where 0 <= t < 1.  Piece 0: p_0 e / e_0 below e_0 (x = 0, w = 1 / e_0);
    // pieces 1 .. n-1: the Hermite cubic of [e_{i-1}, e_i] with end values p and slopes m, in
    // powers of t; piece n: linear with the end slope above e_{n-1}, with w = 2^-60 so that
    // t < 1 far beyond any state (the scaling by a power of two is exact).
    std::vector<double> rec(6 * ((size_t)n_tab + 1));
    auto put = [&](int k, double x, double w, double y, double c1, double c2, double c3) {
        double* r = &rec[6 * (size_t)k];
        r[0] = x; r[1] = w; r[2] = y; r[3] = c1; r[4] = c2; r[5] = c3;
    };
    put(0, 0.0, 1.0 / e_tab[0], 0.0, p_tab[0], 0.0, 0.0);
    for (int i = 1; i < n_tab; i++) {
        const double h = e_tab[i] - e_tab[i - 1];
        const double y0 = p_tab[i - 1], y1 = p_tab[i];
        const double c1 = h * m[i - 1];
        const double c2 = 3.0 * (y1 - y0) - h * (2.0 * m[i - 1] + m[i]);
        const double c3 = 2.0 * (y0 - y1) + h * (m[i - 1] + m[i]);
        put(i, e_tab[i - 1], 1.0 / h, y0, c1, c2, c3);
    }
    put(n_tab, e_tab[n_tab - 1], 0x1p-60, p_tab[n_tab - 1], m[n_tab - 1] * 0x1p60, 0.0, 0.0);
    // log-uniform nodes: the interval comes from log2(e) and a +-1 fix-up
    const double l0 = std::log2(e_tab[0]), l1 = std::log2(e_tab[n_tab - 1]);
    const double dl = (l1 - l0) / (n_tab - 1);
    bool log_uniform = true;
    for (int i = 0; i < n_tab && log_uniform; i++)
        log_uniform = std::fabs(std::log2(e_tab[i]) - (l0 + i * dl)) <= 1e-6 * dl;
    MF_HIP(hipStreamSynchronize(g->stream));
    g->release(g->table_dev);
    g->table_dev = nullptr;
    g->release(g->seed_params);
    g->seed_params = nullptr;
    g->release(g->seed_grid);
    g->seed_grid = nullptr;
    g->has_seed = false;
    int rc = g->alloc(&g->table_dev, rec.size() * sizeof(double));
    if (rc) return rc;
    MF_HIP(hipMemcpy(g->table_dev, rec.data(), rec.size() * sizeof(double), hipMemcpyHostToDevice));
    EosTable& t = g->table;
    t.rec = (const double2*)g->table_dev;
    t.n = n_tab;
    t.log_uniform = log_uniform ? 1 : 0;
    t.lg0 = (float)(l0 - dl);  // piece k + 1 starts at node k
    t.inv_dlg = (float)(1.0 / dl);
    t.seed = nullptr;
    g->eos_kind = MF_EOS_TABLE;
    if (s) {
        int rc2 = install_seed(g, *s);
        if (rc2) return rc2;
    }
    return MF_OK;
}

int mf_set_source_jet(mf_grid_t g, int32_t event, const double x0[3], double v, double dEdx, double sigma)
{
    if (!g || !x0) return fail(MF_ERR_ARG, "null argument");
    if (event < 0 || event >= (int)g->ev.size()) return fail(MF_ERR_ARG, "event out of range");
    if (!(v > 0.0 && v < 1.0) || !(sigma > 0.0) || !std::isfinite(dEdx))
        return fail(MF_ERR_ARG, "jet needs 0 < v < 1, sigma > 0, finite dEdx");
    Event& ev = g->ev[event];
    if (ev.nc == 5 && dEdx != 0.0) return fail(MF_ERR_ARG, "the jet source runs without the charge");
    ev.jet = dEdx != 0.0;
    for (int q = 0; q < 3; q++) ev.jet_x0[q] = x0[q];
    ev.jet_v = v;
    ev.jet_dedx = dEdx;
    ev.jet_sigma = sigma;
    return MF_OK;
}

int mf_set_time(mf_grid_t g, int32_t event, double t, int64_t steps)
{
    if (!g) return fail(MF_ERR_ARG, "null handle");
    if (event < 0 || event >= (int)g->ev.size()) return fail(MF_ERR_ARG, "event out of range");
    if (!std::isfinite(t) || steps < 0) return fail(MF_ERR_ARG, "bad time");
    g->ev[event].t = t;
    g->ev[event].steps = steps;
    return MF_OK;
}

int mf_set_profiling(mf_grid_t g, int32_t enable)
{
    if (!g) return fail(MF_ERR_ARG, "null handle");
    g->profiling = enable != 0;
    return MF_OK;
}

int mf_get_profile(mf_grid_t g, double ms[3], int64_t launches[3])
{
    if (!g || !ms || !launches) return fail(MF_ERR_ARG, "null argument");
    MF_HIP(hipStreamSynchronize(g->stream));
    for (int q = 0; q < 3; q++) {
        ms[q] = 0.0;
        launches[q] = 0;
    }
    for (auto& t : g->timed) {
        float dt = 0.0f;
        MF_HIP(hipEventElapsedTime(&dt, t.start, t.stop));
        ms[t.axis] += dt;
        launches[t.axis]++;
        g->pool.push_back(t.start);
        g->pool.push_back(t.stop);
    }
    g->timed.clear();
    return MF_OK;
}

int mf_set_tuning(mf_grid_t g, const int32_t seg[3], int32_t block)
{
    if (!g) return fail(MF_ERR_ARG, "null handle");
    if (block != 64 && block != 128 && block != 256) return fail(MF_ERR_ARG, "block must be 64, 128 or 256");
    for (int q = 0; q < 3; q++) {
        if (seg && seg[q] < 0) return fail(MF_ERR_ARG, "seg must be >= 0");
        g->seg_override[q] = seg ? seg[q] : 0;
    }
    g->block = block;
    return MF_OK;
}

static int check_strict(mf_grid_t g, const mf_stats* st);

static int collect_stats(mf_grid_t g, const double* dts, mf_stats* st)
{
    const int ne = (int)g->ev.size();
    for (int i = 0; i < ne; i++) {
        int rc = enqueue_totals_any(g->stream, g->dpartial, g->ev[i], g->dtot + (size_t)kMaxComp * i);
        if (rc) return rc;
    }
    std::vector<unsigned long long> hs((size_t)ST_WORDS * ne);
    std::vector<double> ht((size_t)kMaxComp * ne);
    MF_HIP(hipMemcpyAsync(hs.data(), g->dstats, hs.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                          g->stream));
    MF_HIP(hipMemcpyAsync(ht.data(), g->dtot, ht.size() * sizeof(double), hipMemcpyDeviceToHost, g->stream));
    MF_HIP(hipStreamSynchronize(g->stream));
    for (int i = 0; i < ne; i++)
        fill_stats(g->ev[i], &hs[(size_t)ST_WORDS * i], &ht[(size_t)kMaxComp * i], dts[i], st[i]);
    return MF_OK;
}

int mf_step(mf_grid_t g, double dt, int32_t nsteps, mf_stats* st)
{
    if (!g) return fail(MF_ERR_ARG, "null handle");
    if (g->eos_kind < 0) return fail(MF_ERR_STATE, "no equation of state set");
    if (!(dt > 0.0) || !std::isfinite(dt)) return fail(MF_ERR_ARG, "dt must be finite and > 0");
    if (nsteps < 0) return fail(MF_ERR_ARG, "nsteps must be >= 0");
    const int ne = (int)g->ev.size();
    hipError_t e = launch_fill_u64(g->stream, g->dstats, (int64_t)ST_WORDS * ne, 0ULL);
    if (e != hipSuccess) return fail(MF_ERR_HIP, std::string("stats reset: ") + hipGetErrorString(e));
    for (int i = 0; i < ne; i++) {
        Event& ev = g->ev[i];
        unsigned long long* stats = g->dstats + (size_t)ST_WORDS * i;
        int rc = run_steps(g, ev, stats, dt, nsteps);
        if (rc) return rc;
    }
    bool strict = false;
    for (const Event& ev : g->ev) strict = strict || (ev.d.flags & MF_FLAG_STRICT);
    if (!st && !strict) return MF_OK;
    std::vector<mf_stats> local;
    if (!st) {
        local.resize(ne);
        st = local.data();
    }
    std::vector<double> dts(ne, dt);
    int rc = collect_stats(g, dts.data(), st);
    if (rc) return rc;
    return check_strict(g, st);
}

static int check_strict(mf_grid_t g, const mf_stats* st)
{
    const int ne = (int)g->ev.size();
    for (int i = 0; i < ne; i++) {
        const int rc = strict_status(g->ev[i].d, st[i], i);
        if (rc) return rc;
    }
    return MF_OK;
}

int mf_batch_step(mf_grid_t g, const double* dt, int32_t nsteps, mf_stats* st)
{
    if (!g || !dt) return fail(MF_ERR_ARG, "null argument");
    if (g->eos_kind < 0) return fail(MF_ERR_STATE, "no equation of state set");
    if (nsteps < 0) return fail(MF_ERR_ARG, "nsteps must be >= 0");
    const int ne = (int)g->ev.size();
    for (int i = 0; i < ne; i++) {
        if (!(dt[i] > 0.0) || !std::isfinite(dt[i])) return fail(MF_ERR_ARG, "dt must be finite and > 0");
        const mf_grid_desc& d0 = g->ev[0].d;
        const mf_grid_desc& di = g->ev[i].d;
        if (di.dtype != d0.dtype || di.limiter != d0.limiter || di.rk_order != d0.rk_order)
            return fail(MF_ERR_ARG, "batched events must share dtype, limiter and rk_order");
        if (di.flags & MF_FLAG_UNSPLIT_HANCOCK)
            return fail(MF_ERR_ARG, "the unsplit Hancock ablation runs with mf_step only");
        if (di.flags & MF_FLAG_CHARGE) return fail(MF_ERR_ARG, "events with the charge run with mf_step only");
    }
    int rc = ensure_batch_buffers(g);
    if (rc) return rc;
    auto& b = g->batch;
    // order after earlier work on the handle's stream
    MF_HIP(hipEventRecord(b.ev_in, g->stream));
    MF_HIP(hipStreamWaitEvent(b.stream, b.ev_in, 0));
    if ((rc = batch_prepare_any(g, dt))) return rc;
    b.t_host.resize(ne);
    for (int i = 0; i < ne; i++) b.t_host[i] = g->ev[i].t;
    MF_HIP(hipMemcpyAsync(b.t_dev, b.t_host.data(), sizeof(double) * ne, hipMemcpyHostToDevice, b.stream));
    hipError_t e = launch_fill_u64(b.stream, g->dstats, (int64_t)ST_WORDS * ne, 0ULL);
    if (e != hipSuccess) return fail(MF_ERR_HIP, std::string("stats reset: ") + hipGetErrorString(e));
    for (int s = 0; s < nsteps; s++) MF_HIP(hipGraphLaunch(b.exec, b.stream));
    MF_HIP(hipEventRecord(b.ev_out, b.stream));
    MF_HIP(hipStreamWaitEvent(g->stream, b.ev_out, 0));
    for (int i = 0; i < ne; i++) {
        Event& ev = g->ev[i];
        for (int s = 0; s < nsteps; s++) ev.t = ev.t + dt[i];
        ev.steps += nsteps;
    }
    bool strict = false;
    for (const Event& ev : g->ev) strict = strict || (ev.d.flags & MF_FLAG_STRICT);
    if (!st && !strict) return MF_OK;
    std::vector<mf_stats> local;
    if (!st) {
        local.resize(ne);
        st = local.data();
    }
    if ((rc = collect_stats(g, dt, st))) return rc;
    return check_strict(g, st);
}

int mf_con2prim(mf_grid_t g, const void* const U[], void* const prim[], int64_t n, int32_t* iters_dev,
                int32_t mode)
{
    if (!g || !U || !prim) return fail(MF_ERR_ARG, "null argument");
    if (g->eos_kind < 0) return fail(MF_ERR_STATE, "no equation of state set");
    if (n < 0) return fail(MF_ERR_ARG, "n must be >= 0");
    if (mode != MF_C2P_PLAIN && mode != MF_C2P_SEEDED && mode != MF_C2P_CONFORMAL)
        return fail(MF_ERR_ARG, "unknown con2prim mode");
    if (mode != MF_C2P_PLAIN && g->eos_kind != MF_EOS_TABLE)
        return fail(MF_ERR_ARG, "seeded con2prim needs the table EoS");
    if (mode == MF_C2P_SEEDED && !g->has_seed) return fail(MF_ERR_ARG, "seeded con2prim needs a surrogate");
    if (n == 0) return MF_OK;
    const int nc = g->ev[0].nc;
    for (int c = 0; c < nc; c++)
        if (!U[c]) return fail(MF_ERR_ARG, "null state pointer");
    for (int c = 0; c < nc + 1; c++)
        if (!prim[c]) return fail(MF_ERR_ARG, "null output pointer");
    unsigned long long* stats = g->dstats + (size_t)ST_WORDS * g->ev.size();
    hipError_t e = launch_fill_u64(g->stream, stats, ST_WORDS, 0ULL);
    if (e != hipSuccess) return fail(MF_ERR_HIP, std::string("stats reset: ") + hipGetErrorString(e));
    if (nc == 5) {  // with the charge: FP64, p = c e or the ideal gas
        C2PArgs<double> a;
        for (int c = 0; c < 5; c++) a.U[c] = (const double*)U[c];
        for (int c = 0; c < 6; c++) a.prim[c] = (double*)prim[c];
        a.iters = iters_dev; a.n = n; a.stats = stats;
        if (g->eos_kind == MF_EOS_GAMMA) e = launch_con2prim_charge<EosGamma>(n, g->stream, a, EosGamma::make(g->gamma));
        else e = launch_con2prim_charge<EosIdeal<double>>(n, g->stream, a, EosIdeal<double>::make(g->cs2));
    } else if (mode != MF_C2P_PLAIN) {
        C2PArgs<double> a;
        for (int c = 0; c < 4; c++) a.U[c] = (const double*)U[c];
        for (int c = 0; c < 5; c++) a.prim[c] = (double*)prim[c];
        a.iters = iters_dev; a.n = n; a.stats = stats;
        EosTable t = g->table;
        t.seed = nullptr;
        SeedNorm nrm = g->seed_norm;
        e = con2prim_seeded(n, g->stream, a, t, g->seed_params, nrm, mode == MF_C2P_SEEDED ? 1 : 2);
    } else if (g->eos_kind == MF_EOS_TABLE) {
        C2PArgs<double> a;
        for (int c = 0; c < 4; c++) a.U[c] = (const double*)U[c];
        for (int c = 0; c < 5; c++) a.prim[c] = (double*)prim[c];
        a.iters = iters_dev; a.n = n; a.stats = stats;
        EosTable t = g->table;
        t.seed = nullptr;  // plain: bracket midpoint start, whether or not a seed is installed
        e = launch_con2prim<double, EosTable>(n, g->stream, a, t);
    } else if (g->ev[0].d.dtype == MF_F32) {
        C2PArgs<float> a;
        for (int c = 0; c < 4; c++) a.U[c] = (const float*)U[c];
        for (int c = 0; c < 5; c++) a.prim[c] = (float*)prim[c];
        a.iters = iters_dev; a.n = n; a.stats = stats;
        const EosIdeal<float> eos = EosIdeal<float>::make(g->cs2);
        e = launch_con2prim<float, EosIdeal<float>>(n, g->stream, a, eos);
    } else {
        C2PArgs<double> a;
        for (int c = 0; c < 4; c++) a.U[c] = (const double*)U[c];
        for (int c = 0; c < 5; c++) a.prim[c] = (double*)prim[c];
        a.iters = iters_dev; a.n = n; a.stats = stats;
        const EosIdeal<double> eos = EosIdeal<double>::make(g->cs2);
        e = launch_con2prim<double, EosIdeal<double>>(n, g->stream, a, eos);
    }
    if (e != hipSuccess) return fail(MF_ERR_HIP, std::string("con2prim launch: ") + hipGetErrorString(e));
    return MF_OK;
}

int mf_con2prim_stats(mf_grid_t g, int64_t out[4])
{
    if (!g || !out) return fail(MF_ERR_ARG, "null argument");
    unsigned long long h[ST_WORDS];
    MF_HIP(hipMemcpyAsync(h, g->dstats + (size_t)ST_WORDS * g->ev.size(), sizeof(h), hipMemcpyDeviceToHost,
                          g->stream));
    MF_HIP(hipStreamSynchronize(g->stream));
    out[0] = (int64_t)h[ST_FLOOR];
    out[1] = (int64_t)h[ST_BAD];
    out[2] = (int64_t)h[ST_ITERS];
    out[3] = (int64_t)h[ST_FALLBACK];
    return MF_OK;
}

int64_t mf_mlp_workspace(int64_t n) { return n > 0 ? mlp_grad_partials(n) * (MF_MLP_PARAMS + 1) : 0; }

int mf_mlp_forward(const float* params, const float* X, int64_t n, float* y, void* stream)
{
    if (!params || n < 0 || (n > 0 && (!X || !y))) return fail(MF_ERR_ARG, "bad argument");
    hipError_t e = mlp_forward(params, X, n, y, (hipStream_t)stream);
    if (e != hipSuccess) return fail(MF_ERR_HIP, std::string("mlp forward: ") + hipGetErrorString(e));
    return MF_OK;
}

int mf_mlp_grad(const float* params, const float* X, const float* t, int64_t n, float* grad, float* loss, float* work,
                int64_t work_floats, void* stream)
{
    if (!params || !X || !t || !grad || !work || n < 1) return fail(MF_ERR_ARG, "bad argument");
    if (work_floats < mf_mlp_workspace(n)) return fail(MF_ERR_ARG, "workspace too small (see mf_mlp_workspace)");
    hipError_t e = mlp_grad(params, X, t, n, work, grad, loss, (hipStream_t)stream);
    if (e != hipSuccess) return fail(MF_ERR_HIP, std::string("mlp grad: ") + hipGetErrorString(e));
    return MF_OK;
}

int mf_mlp_grad_noalloc(const float* params, const float* X, const float* t, int64_t n, float* grad, float* loss,
                        void* stream)
{
    if (!params || !X || !t || !grad || n < 1) return fail(MF_ERR_ARG, "bad argument");
    if (n > MF_MLP_NOALLOC_MAX_N)
        return fail(MF_ERR_ARG, "n = " + std::to_string(n) + " exceeds MF_MLP_NOALLOC_MAX_N = " +
                                    std::to_string(MF_MLP_NOALLOC_MAX_N) + " (use mf_mlp_grad with a workspace)");
    if (mf_mlp_workspace(n) > kNoallocFloats) return fail(MF_ERR_ARG, "scratch array too small for n");
    float* part = nullptr;
    const int rc = noalloc_scratch(&part);
    if (rc != MF_OK) return rc;
    hipError_t e = mlp_grad(params, X, t, n, part, grad, loss, (hipStream_t)stream);
    if (e != hipSuccess) return fail(MF_ERR_HIP, std::string("mlp grad (no-alloc): ") + hipGetErrorString(e));
    return MF_OK;
}

int mf_mlp_adam(float* params, const float* grad, float* m, float* v, int32_t step, float lr, float beta1, float beta2,
                float eps, void* stream)
{
    if (!params || !grad || !m || !v || step < 1 || !(lr > 0.0f)) return fail(MF_ERR_ARG, "bad argument");
    hipError_t e = mlp_adam(params, grad, m, v, step, lr, beta1, beta2, eps, (hipStream_t)stream);
    if (e != hipSuccess) return fail(MF_ERR_HIP, std::string("mlp adam: ") + hipGetErrorString(e));
    return MF_OK;
}

int mf_totals(mf_grid_t g, int32_t event, double* out)
{
    if (!g || !out) return fail(MF_ERR_ARG, "null argument");
    if (event < 0 || event >= (int)g->ev.size()) return fail(MF_ERR_ARG, "event out of range");
    const Event& ev = g->ev[event];
    double* dt = g->dtot + (size_t)kMaxComp * event;
    int rc = enqueue_totals_any(g->stream, g->dpartial, ev, dt);
    if (rc) return rc;
    MF_HIP(hipMemcpyAsync(out, dt, ev.nc * sizeof(double), hipMemcpyDeviceToHost, g->stream));
    MF_HIP(hipStreamSynchronize(g->stream));
    return MF_OK;
}

}  // extern "C"
