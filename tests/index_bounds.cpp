// Host check of the index maps of the axis sweeps (mf_index.hpp): for small
// grids, every element index the y/z march, the x sweep's row stream and the
// unsplit correction pre-pass form -- loads, look-aheads and stores -- lies
// inside its array, and every cell is written exactly once per sweep.  The
// loops follow the kernels' loop bounds (sweep_line, sweep_x_wave,
// k_unsplit_delta in mf_kernels.hip); the index functions are the kernels' own.
//
// Build: g++ -std=c++17 -I paper_1510_06340_amd/csrc tests/index_bounds.cpp
// Prints "ok <checks>" and exits 0, or prints the first violation and exits 1.
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "mf_index.hpp"

using mf::ghost;
using mf::march_ahead;
using mf::x_item;

static long long g_checks = 0;

static void check(bool ok, const char* what, long long a, long long b, long long c, long long d)
{
    g_checks++;
    if (!ok) {
        std::printf("FAIL %s: %lld %lld %lld %lld\n", what, a, b, c, d);
        std::exit(1);
    }
}

// ghost() is the boundary rule: outflow clamps, periodic wraps, on [-2, N+1].
static void check_ghost_rule()
{
    for (int N = 1; N <= 8; N++)
        for (int j = -2; j <= N + 1; j++) {
            const int o = ghost(j, N, 0), p = ghost(j, N, 1);
            check(o == (j < 0 ? 0 : (j >= N ? N - 1 : j)), "outflow rule", N, j, o, 0);
            check(p == ((j % N) + N) % N, "periodic rule", N, j, p, 0);
        }
}

// The y/z march of every segment of one line: loads at ghost indices, stores
// at the segment's own cells.  dl: the unsplit sweeps also read the extended
// coordinate j + 2 of the corrections (N + 2 cells).
static void check_march(int N, int periodic, int seg)
{
    std::vector<int> written(N, 0);
    for (int s0 = 0; s0 < N; s0 += seg) {
        const int s1 = s0 + seg < N ? s0 + seg : N;
        for (int pre = s0 - 2; pre <= s0; pre++) {
            const int g = ghost(pre, N, periodic);
            check(g >= 0 && g < N, "march preload", N, periodic, seg, pre);
        }
        for (int j = s0 - 2; j < s1; j++) {
            const int g = ghost(march_ahead(j, N), N, periodic);
            check(g >= 0 && g < N, "march look-ahead", N, periodic, seg, j);
            // a look-ahead that is used (not the last iteration) is the unclamped cell j + 3
            if (j + 1 < s1) check(march_ahead(j, N) == j + 3, "look-ahead value", N, periodic, seg, j);
            const int ext = j + 2;
            check(ext >= 0 && ext < N + 2, "unsplit extended coordinate", N, periodic, seg, j);
            if (j >= s0) {
                check(j < N, "march store", N, periodic, seg, j);
                written[j]++;
            }
        }
    }
    for (int i = 0; i < N; i++) check(written[i] == 1, "march writes each cell once", N, periodic, seg, i);
}

// The x sweep over nlines rows of N cells, wavefronts of 64 lanes taking
// 64 * seg consecutive items each, starting two items early.
static void check_x_sweep(int N, int periodic, long long nlines, int seg, int nx, int ny, int nz)
{
    const long long P = (long long)N + 2;
    const long long total = nlines * P;
    const long long ncell = nlines * N;
    std::vector<int> written(ncell, 0);
    for (long long wave = 0;; wave++) {
        const long long s = wave * 64 * (long long)seg;
        if (s >= total) break;
        const long long e = s + 64LL * seg < total ? s + 64LL * seg : total;
        int64_t row[64];
        int x[64];
        for (int lane = 0; lane < 64; lane++) {
            const long long it = s - 2 + lane;
            if (it >= 0) {
                x_item(it, N, row[lane], x[lane]);
            } else {
                x[lane] = (int)(it + P) - 1;
                row[lane] = -1;
            }
        }
        for (long long c0 = s - 2; c0 < e; c0 += 64) {
            bool edge = false;
            long long base[64];
            int xc[64];
            bool valid[64];
            for (int lane = 0; lane < 64; lane++) {
                const long long it = c0 + lane;
                valid[lane] = it >= 0 && it < e;
                base[lane] = (valid[lane] ? row[lane] : 0) * (long long)N;
                xc[lane] = valid[lane] ? x[lane] : 0;
                edge = edge || !valid[lane] || xc[lane] < 1 || xc[lane] > N - 2;
                if (valid[lane]) {
                    int64_t r2;
                    int x2;
                    x_item(it, N, r2, x2);
                    check(r2 == row[lane] && x2 == x[lane], "x stream position", N, nlines, seg, it);
                }
            }
            for (int lane = 0; lane < 64; lane++) {
                const long long it = c0 + lane;
                if (!edge) {
                    for (int o = -1; o <= 1; o++) {
                        const long long i = base[lane] + xc[lane] + o;
                        check(i >= 0 && i < ncell, "x fast-path load", N, nlines, seg, it);
                    }
                } else {
                    for (int o = -1; o <= 1; o++) {
                        const long long i = base[lane] + ghost(xc[lane] + o, N, periodic);
                        check(i >= 0 && i < ncell, "x ghost load", N, nlines, seg, it);
                    }
                }
                // unsplit corrections of the lane's cell in the extended grid
                if (nx == N) {
                    const long long r = valid[lane] ? row[lane] : 0;
                    const long long es_f = nx + 2, es_s = (long long)(nx + 2) * (ny + 2);
                    const long long ei = (long long)(xc[lane] + 1) + (r % ny + 1) * es_f + (r / ny + 1) * es_s;
                    check(ei >= 0 && ei < (long long)(nx + 2) * (ny + 2) * (nz + 2), "x unsplit load", N, nlines,
                          seg, it);
                }
                if (valid[lane] && x[lane] >= 1 && it >= s) {
                    const long long ij = base[lane] + (x[lane] - 1);
                    check(ij >= 0 && ij < ncell, "x store", N, nlines, seg, it);
                    written[ij]++;
                }
            }
            for (int lane = 0; lane < 64; lane++) {
                x[lane] += 64;
                while (x[lane] > N) {
                    x[lane] -= (int)P;
                    row[lane]++;
                }
            }
        }
    }
    for (long long i = 0; i < ncell; i++) check(written[i] == 1, "x writes each cell once", N, nlines, seg, i);
}

// The unsplit pre-pass: one thread per column of the extended grid, marching
// zseg extended planes; loads of the cell and its six neighbours.
static void check_unsplit_prepass(const int n[3], const int per[3], int zseg)
{
    const long long ex = n[0] + 2, ey = n[1] + 2;
    const int ez = n[2] + 2;
    const long long ncell = (long long)n[0] * n[1] * n[2];
    const long long sy = n[0], sz = (long long)n[0] * n[1];
    std::vector<int> written(ex * ey * ez, 0);
    for (long long col = 0; col < ex * ey; col++)
        for (int z0 = 0; z0 < ez; z0 += zseg) {
            const int z1 = z0 + zseg < ez ? z0 + zseg : ez;
            const long long row = col / ex;
            const int q0 = (int)(col - row * ex) - 1, q1 = (int)row - 1;
            const int g0 = ghost(q0, n[0], per[0]), g1 = ghost(q1, n[1], per[1]);
            const long long cxy = g0 + sy * g1;
            const long long off[4] = {ghost(q0 - 1, n[0], per[0]) - g0, ghost(q0 + 1, n[0], per[0]) - g0,
                                      sy * (ghost(q1 - 1, n[1], per[1]) - g1),
                                      sy * (ghost(q1 + 1, n[1], per[1]) - g1)};
            auto plane = [&](int q2) { return cxy + sz * ghost(q2, n[2], per[2]); };
            for (int q2 = z0 - 2; q2 <= z0 - 1; q2++)
                check(plane(q2) >= 0 && plane(q2) < ncell, "pre-pass preload", n[0], n[1], n[2], col);
            for (int ze = z0; ze < z1; ze++) {
                const long long i0 = plane(ze - 1);
                check(plane(ze) >= 0 && plane(ze) < ncell, "pre-pass z load", n[0], n[1], n[2], col);
                for (int q = 0; q < 4; q++)
                    check(i0 + off[q] >= 0 && i0 + off[q] < ncell, "pre-pass x/y load", n[0], n[1], n[2], col);
                written[col + (long long)ze * ex * ey]++;
            }
        }
    for (size_t i = 0; i < written.size(); i++)
        check(written[i] == 1, "pre-pass writes each extended cell once", n[0], n[1], n[2], (long long)i);
}

int main()
{
    check_ghost_rule();
    for (int N = 1; N <= 9; N++)
        for (int periodic = 0; periodic <= 1; periodic++)
            for (int seg = 1; seg <= N + 3; seg++) check_march(N, periodic, seg);
    // the unclamped look-ahead of the last iteration leaves [0, N) on a 2-cell periodic line
    // (the out-of-bounds read this map removes): keep the check sensitive to it
    {
        const int N = 2, j = N - 1;
        const int g = ghost(j + 3, N, 1);
        check(!(g >= 0 && g < N), "unclamped look-ahead is out of range (sensitivity)", N, j, g, 0);
    }
    const int ns[] = {1, 2, 3, 4, 5, 6, 7, 62, 63, 64, 65, 130};
    for (int N : ns)
        for (int periodic = 0; periodic <= 1; periodic++)
            for (long long nl : {1LL, 2LL, 3LL, 5LL, 7LL})
                for (int seg : {1, 2, 3})
                    check_x_sweep(N, periodic, nl, seg, N, (int)nl, 1);
    // x sweep rows of a (nx, ny, nz) grid: line r = y + ny z
    for (int nx : {1, 2, 5, 66})
        for (int ny : {1, 2, 3})
            for (int nz : {1, 2, 4})
                for (int periodic = 0; periodic <= 1; periodic++)
                    check_x_sweep(nx, periodic, (long long)ny * nz, 2, nx, ny, nz);
    for (int a : {1, 2, 3})
        for (int b : {1, 2, 5})
            for (int c : {1, 2, 3, 9})
                for (int pm = 0; pm < 8; pm++) {
                    const int n[3] = {a, b, c}, per[3] = {pm & 1, (pm >> 1) & 1, (pm >> 2) & 1};
                    for (int zseg : {1, 3, 8}) check_unsplit_prepass(n, per, zseg);
                }
    std::printf("ok %lld\n", g_checks);
    return 0;
}
