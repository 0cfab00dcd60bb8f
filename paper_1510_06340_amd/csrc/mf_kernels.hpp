// mf_kernels.hpp -- host-side launchers of the gfx950 kernels (mf_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "mf_device.hpp"
#include "mf_params.hpp"

namespace mf {

// One axis sweep of a Runge-Kutta stage; grid = (ceil(nlines / block), nseg).
template <typename T>
hipError_t launch_sweep(int axis, int lim, bool jet, dim3 grid, dim3 block, hipStream_t s,
                        const SweepArgs<T>& a, const EosIdeal<T>& eos);

template <typename T>
hipError_t launch_con2prim(int64_t n, hipStream_t s, const C2PArgs<T>& a, const EosIdeal<T>& eos);

// Deterministic sums of the four components over a.n cells, times dV, into out[4] (device).
template <typename T>
hipError_t launch_totals(hipStream_t s, const TotalsArgs<T>& a, int nblocks, double dV, double* out);

hipError_t launch_fill_u64(hipStream_t s, unsigned long long* p, int64_t n, unsigned long long v);

}  // namespace mf
