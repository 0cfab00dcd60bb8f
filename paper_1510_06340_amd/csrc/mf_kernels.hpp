// mf_kernels.hpp -- host-side launchers of the gfx950 kernels (mf_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "mf_device.hpp"
#include "mf_params.hpp"

namespace mf {

// One axis sweep of a Runge-Kutta stage; grid = (ceil(nlines / block), nseg).
// Eos = EosIdeal<T> or (T = double) EosTable.
template <typename T, class Eos>
hipError_t launch_sweep(int axis, int lim, bool jet, dim3 grid, dim3 block, hipStream_t s,
                        const SweepArgs<T>& a, const Eos& eos);

template <typename T, class Eos>
hipError_t launch_con2prim(int64_t n, hipStream_t s, const C2PArgs<T>& a, const Eos& eos);

// The MF_FLAG_UNSPLIT_HANCOCK ablation: the three-axis Hancock corrections of
// the stage input over the extended grid (one launch per stage), and the axis
// sweeps that add them to the faces (a.dl and the extended strides set).
template <typename T, class Eos>
hipError_t launch_unsplit_delta(int lim, hipStream_t s, const UnsplitArgs<T>& a, const Eos& eos);
template <typename T, class Eos>
hipError_t launch_sweep_unsplit(int axis, int lim, bool jet, dim3 grid, dim3 block, hipStream_t s,
                                const SweepArgs<T>& a, const Eos& eos);

// Resident wavefronts per SIMD of the sweep kernel along axis (the z kernel
// with the jet source when jet), from its register and LDS use, at the given
// block size.
template <typename T, class Eos>
int sweep_waves_per_simd(int axis, int lim, bool jet, int block);

// Deterministic sums of the nc (4 or 5) components over a.n cells, times dV, into out[nc] (device);
// a.partial holds kMaxComp doubles per block.
template <typename T>
hipError_t launch_totals(hipStream_t s, const TotalsArgs<T>& a, int nc, int nblocks, double dV, double* out);

// With the conserved charge R (five components; FP64, per event, no jet and
// no unsplit ablation): Eos = EosIdeal<double> (a passive charge) or EosGamma.
template <class Eos>
hipError_t launch_sweep_charge(int axis, int lim, dim3 grid, dim3 block, hipStream_t s, const SweepArgs<double>& a,
                               const Eos& eos);
template <class Eos>
int sweep_waves_per_simd_charge(int axis, int lim, int block);
// con2prim of n states with the charge: a.U has 5 arrays, a.prim 6 (n = R sqrt(1 - v^2) last).
template <class Eos>
hipError_t launch_con2prim_charge(int64_t n, hipStream_t s, const C2PArgs<double>& a, const Eos& eos);

hipError_t launch_fill_u64(hipStream_t s, unsigned long long* p, int64_t n, unsigned long long v);
hipError_t launch_fill_u32(hipStream_t s, unsigned int* p, int n, unsigned int v);

// One batched axis sweep: a persistent grid (resident blocks of the device)
// draining the tile queue described by tab (one SweepArgs per event) and
// tile_start (ne + 1 prefix offsets); *counter must be 0.
template <typename T, class Eos>
hipError_t launch_batch_sweep(int axis, int lim, bool jet, const SweepArgs<T>* tab, const int64_t* tile_start, int ne,
                              unsigned int* counter, int64_t total_tiles, int block, hipStream_t s, const Eos& eos);

// t[i] += dt[i], i < ne (device event times of batched stepping).
hipError_t launch_advance_time(hipStream_t s, double* t, const double* dt, int ne);

}  // namespace mf
