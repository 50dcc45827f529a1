// Launchers of the differentiation-form kernels (step adjoint, moment adjoint); the
// recording forward step is declared beside the other step launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rsol_launch.hpp"
#include "rsol_sort.hpp"

namespace rsol {

// LDS slots per field component of the region the tiled kernels of the differentiation
// form stage (a 4x4x4 tile with a two-cell halo, laid out by region_index).
constexpr int kAdjRegion = 600;

// Layout of a staged region of rx x ry x rz cells: x fastest, rows of rx, planes padded
// to a pitch of 12 (mod 32) elements.  A wave's 64 lanes hold packets of the 64 cells of
// one tile (the sort orders a tile rank-major); with planes of 64 elements the four
// z-layers of the tile would fall on the same LDS banks.
__host__ __device__ inline int region_plane_pitch(int rx, int ry) {
  const int p = rx * ry;
  return p + ((12 - p % 32) % 32 + 32) % 32;
}
__host__ __device__ inline int region_index(int ax, int ay, int az, int rx, int pz) { return ax + rx * ay + pz * az; }
// Slots a region of rx x ry x rz cells spans.
__host__ __device__ inline int region_span(int rx, int ry, int rz) {
  return region_plane_pitch(rx, ry) * (rz - 1) + rx * ry;
}

// Reverse of one step whose starting state is in `slab`: lam_x, lam_u [3][np] hold
// dL/d(state after) on entry and dL/d(state before) on exit; gE, gB [3][n_cells] and
// accumulate; lam_dM [3][n_cells] / lam_dE [n_cells] (optional) are the cotangents of
// the step's exchange deposit.
template <typename T>
hipError_t launch_step_backward(int shape, const void* slab, int64_t np, T* lam_x, T* lam_u, const T* E, const T* B,
                                const double* lam_dM, const double* lam_dE, double* gE, double* gB,
                                const RunConsts& k, hipStream_t s);

// Same reverse step with the packets held in tile order: tile t's packets are entries
// [offsets[t*cells_per_tile], offsets[(t+1)*cells_per_tile]) of slab, lam_x and lam_u,
// as a counting sort of this step's starting state or of one a few steps earlier leaves
// them.  dL/dE, dL/dB accumulate per tile in LDS over the tile plus a halo of `halo`
// cells; packets outside it are listed in `spill` (np + 2 int32 of scratch: two counts,
// then indices; this step counts in spill[parity]), and launch_step_backward_spilled
// reverses them with global atomics.  launch_spill_clear zeroes both counts before the
// first step of a sweep; each spilled launch zeroes the count the next step uses.
// Needs step_backward_tiled_fits(t, halo).
bool step_backward_tiled_fits(const Tiling& t, int halo);
hipError_t launch_iota(int32_t* p, int64_t n, hipStream_t s);
hipError_t launch_spill_clear(int32_t* spill, hipStream_t s);
template <typename T>
hipError_t launch_step_backward_tiled(int shape, const Packets<T>& slab, const int32_t* offsets,
                                      const Tiling& t, int halo, int32_t* spill, int parity, T* lam, const T* E,
                                      const T* B, const double* lam_dM, const double* lam_dE, double* gE,
                                      double* gB, const RunConsts& k, hipStream_t s);
template <typename T>
hipError_t launch_step_backward_spilled(int shape, const Packets<T>& slab, int32_t* spill, int parity, T* lam,
                                        const T* E, const T* B, const double* lam_dM, const double* lam_dE,
                                        double* gE, double* gB, const RunConsts& k, hipStream_t s);

// The tile-ordered sweeps hold the adjoints as records of six values per packet (dL/dx
// then dL/du, 6 * np values).  launch_permute_records: dst[j] = src[idx[j]] (records;
// idx a permutation of 0..np-1).  launch_records_rows: the caller's lam_x [3][np],
// lam_u [3][np] into records in a tile order, rec[j] = packet order[j], or back into
// the caller's arrays with to_rows; tmp holds 6 * np values of work space.
template <typename T>
hipError_t launch_permute_records(const T* src, T* dst, const int32_t* idx, int64_t np, hipStream_t s);
template <typename T>
hipError_t launch_records_rows(T* lam_x, T* lam_u, T* rec, T* tmp, const int32_t* order, int64_t np, bool to_rows,
                               hipStream_t s);

// Packets held in tile order back into the caller's arrays: P[S.id[j]] = S[j]
// (positions and momenta).
template <typename T>
hipError_t launch_unsort(const Packets<T>& S, const Packets<T>& P, hipStream_t s);

// Adjoint of the moment deposit at the current state, added into lam_x, lam_u.
template <typename T>
hipError_t launch_moments_backward(int shape, const Packets<T>& P, const double* lrho, const double* lP,
                                   const double* le, T* lam_x, T* lam_u, const RunConsts& k, hipStream_t s);

}  // namespace rsol
