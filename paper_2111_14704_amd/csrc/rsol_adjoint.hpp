// Launchers of the differentiation-form kernels (step adjoint, moment adjoint); the
// recording forward step is declared beside the other step launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rsol_launch.hpp"
#include "rsol_sort.hpp"

namespace rsol {

// Reverse of one step whose starting state is in `slab`: lam_x, lam_u [3][np] hold
// dL/d(state after) on entry and dL/d(state before) on exit; gE, gB [3][n_cells] and
// accumulate; lam_dM [3][n_cells] / lam_dE [n_cells] (optional) are the cotangents of
// the step's exchange deposit.
template <typename T>
hipError_t launch_step_backward(int shape, const void* slab, int64_t np, T* lam_x, T* lam_u, const T* E, const T* B,
                                const double* lam_dM, const double* lam_dE, double* gE, double* gB,
                                const RunConsts& k, hipStream_t s);

// Same reverse step with the packets taken tile by tile: `order` (packet indices in the
// recorded order, tile by tile) and `offsets` (first entry of each tile) come from a
// counting sort (launch_sort with the packets' recorded indices as ids) of this step's
// starting state or of one a few steps later; `slab` is this step's starting state in
// the recorded order.  dL/dE, dL/dB accumulate per tile in LDS over the tile plus a halo
// of `halo` cells; packets outside it are listed in `spill` (np + 1 int32 of scratch)
// and reversed by a second kernel with global atomics.  Needs
// step_backward_tiled_fits(t, halo).
bool step_backward_tiled_fits(const Tiling& t, int halo);
hipError_t launch_iota(int32_t* p, int64_t n, hipStream_t s);
template <typename T>
hipError_t launch_step_backward_tiled(int shape, const Packets<T>& slab, const int32_t* order, const int32_t* offsets,
                                      const Tiling& t, int halo, int32_t* spill, T* lam_x, T* lam_u, const T* E,
                                      const T* B, const double* lam_dM, const double* lam_dE, double* gE, double* gB,
                                      const RunConsts& k, hipStream_t s);

// Adjoint of the moment deposit at the current state, added into lam_x, lam_u.
template <typename T>
hipError_t launch_moments_backward(int shape, const Packets<T>& P, const double* lrho, const double* lP,
                                   const double* le, T* lam_x, T* lam_u, const RunConsts& k, hipStream_t s);

}  // namespace rsol
