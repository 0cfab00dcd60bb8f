// mf_index.hpp -- index maps of the axis sweeps: ghost cells and the march
// look-ahead.  Host and device: the kernels use them, and a host program
// enumerates every index they form for small grids and checks that it stays
// inside the arrays.
#pragma once

#include <stdint.h>

#if defined(__HIPCC__)
#define MF_HD __host__ __device__
#else
#define MF_HD
#endif

namespace mf {

// Ghost cells along a line of N cells, two per side: outflow copies the edge
// cell, periodic wraps.  Defined for j in [-2, N+1] (N >= 2 needs one wrap;
// N == 1 maps every index to 0); the result is in [0, N).
MF_HD inline int ghost(int j, int N, int periodic)
{
    if (periodic) return (N == 1) ? 0 : (j < 0 ? j + N : (j >= N ? j - N : j));
    return j < 0 ? 0 : (j >= N ? N - 1 : j);
}

// Cell loaded one step ahead by iteration j of the y/z march over a segment
// [s0, s1) of a line of N cells (s0 - 2 <= j < s1; iteration j works on
// cells j .. j+2 and loads cell j + 3 for the next one), clamped to the last
// ghost cell N + 1.  Only the last iteration of a segment ending at N
// (j = N - 1) is clamped, and the value it loads is never used.
MF_HD inline int march_ahead(int j, int N) { return j + 3 <= N + 1 ? j + 3 : N + 1; }

// Item `it` >= 0 of the x sweep's row stream: rows of N + 2 items, item
// (row, x) for x = -1..N.
MF_HD inline void x_item(int64_t it, int N, int64_t& row, int& x)
{
    const int64_t P = (int64_t)N + 2;
    row = it / P;
    x = (int)(it - row * P) - 1;
}

}  // namespace mf
