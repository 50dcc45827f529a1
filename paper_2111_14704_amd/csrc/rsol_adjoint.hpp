// Launchers of the differentiation-form kernels (forward state recording, step
// adjoint, moment adjoint).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rsol_launch.hpp"
#include "rsol_sort.hpp"

namespace rsol {

// Copy the current packet state into a state slab: FP64 form [6][np] doubles
// (x0, x1, x2, u0, u1, u2); FP32 form [7][np] 4-byte words (cell, off0..2, u0..2).
template <typename T>
hipError_t launch_record(const Packets<T>& P, void* slab, hipStream_t s);

// Reverse of one step whose starting state is in `slab`: lam_x, lam_u [3][np] hold
// dL/d(state after) on entry and dL/d(state before) on exit; gE, gB [3][n_cells] and
// accumulate; lam_dM [3][n_cells] / lam_dE [n_cells] (optional) are the cotangents of
// the step's exchange deposit.
template <typename T>
hipError_t launch_step_backward(int shape, const void* slab, int64_t np, T* lam_x, T* lam_u, const T* E, const T* B,
                                const double* lam_dM, const double* lam_dE, double* gE, double* gB,
                                const RunConsts& k, hipStream_t s);

// Same reverse step with the starting state counting-sorted by tile (launch_sort of the
// slab with id = the packets' recorded indices into `sorted`, offsets = the sort's bin
// offsets): dL/dE, dL/dB accumulate per tile in LDS.  Needs a tiling whose tile plus a
// one-cell halo fits the LDS region (step_backward_tiled_fits).
bool step_backward_tiled_fits(const Tiling& t);
hipError_t launch_iota(int32_t* p, int64_t n, hipStream_t s);
template <typename T>
hipError_t launch_step_backward_tiled(int shape, const Packets<T>& sorted, const int32_t* offsets, const Tiling& t,
                                      T* lam_x, T* lam_u, const T* E, const T* B, const double* lam_dM,
                                      const double* lam_dE, double* gE, double* gB, const RunConsts& k,
                                      hipStream_t s);

// Adjoint of the moment deposit at the current state, added into lam_x, lam_u.
template <typename T>
hipError_t launch_moments_backward(int shape, const Packets<T>& P, const double* lrho, const double* lP,
                                   const double* le, T* lam_x, T* lam_u, const RunConsts& k, hipStream_t s);

}  // namespace rsol
