// Host-side launchers of the library's kernels.  Every launcher enqueues work
// on the given stream and returns the launch status; none synchronises.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rsol_particles.hpp"

namespace rsol {

constexpr int kShapeCIC = 1;
constexpr int kShapeTSC = 2;

// Gas side of a coupled step (density and magnetic field held fixed, no MHD solver).
// The step's exchange is added into the gas momentum mom and energy egas (Eq. (12));
// afterwards every cell refreshes u_gas = mom/rho and E = -(u_gas/c) x B with the true
// c (Sec. 2, after Eq. (5)), writing E and, in the FP32 form, its float copy.
struct GasLink {
  const double* rho;  // [n_cells] gas density; NULL when the step is not coupled
  double* mom;        // [3][n_cells] gas momentum density rho u (the step's dM)
  double* egas;       // [n_cells] gas energy density (the step's dE), may be NULL
  const double* B;    // [3][n_cells]
  double* E;          // [3][n_cells] out
  float* E32;         // [3][n_cells] FP32 copy of E, or NULL
  double inv_c;       // 1/c
};

// E of one cell from its gas momentum (the refresh of a coupled step).
__device__ __forceinline__ void gas_refresh(const GasLink& g, int64_t c, int64_t nc) {
  const double r = g.rho[c];
  const double ux = g.mom[c] / r, uy = g.mom[nc + c] / r, uz = g.mom[2 * nc + c] / r;
  const double bx = g.B[c], by = g.B[nc + c], bz = g.B[2 * nc + c];
  const double ex = -(uy * bz - uz * by) * g.inv_c;
  const double ey = -(uz * bx - ux * bz) * g.inv_c;
  const double ez = -(ux * by - uy * bx) * g.inv_c;
  g.E[c] = ex;
  g.E[nc + c] = ey;
  g.E[2 * nc + c] = ez;
  if (g.E32) {
    g.E32[c] = (float)ex;
    g.E32[nc + c] = (float)ey;
    g.E32[2 * nc + c] = (float)ez;
  }
}

// fields and conversions
hipError_t launch_gas_field(const GasLink& g, int64_t ncells, hipStream_t s);
hipError_t launch_electric_field(const double* u_gas, const double* B, double* E, int ncells,
                                 double c, hipStream_t s);
hipError_t launch_to_fp32(const double* src, float* dst, int64_t n, hipStream_t s);
hipError_t launch_positions_to_cells(const double* x, int32_t* cell, float* off, int64_t np,
                                     const RunConsts& k, hipStream_t s);
hipError_t launch_cells_to_positions(const int32_t* cell, const float* off, double* x, int64_t np,
                                     const RunConsts& k, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t s);

// timestep inputs: out[0] = max beta (bits), out[1] = min gamma (bits), out[2] = max |B| (bits),
// out[3] = max nucleon density (bits; 0 when nn is NULL)
template <typename T>
hipError_t launch_dt_inputs(const Packets<T>& P, const double* B, const double* nn, int ncells,
                            unsigned long long* out, hipStream_t s);

// unfused phases (one thread per packet, any packet order)
template <typename T>
hipError_t launch_gather(int shape, const Packets<T>& P, const T* E, const T* B, T* Ep, T* Bp,
                         const RunConsts& k, hipStream_t s);
template <typename T>
hipError_t launch_push(const Packets<T>& P, const T* Ep, const T* Bp, T* payload,
                       const RunConsts& k, hipStream_t s);
template <typename T>
hipError_t launch_deposit(int shape, const Packets<T>& P, const T* payload, double* dM, double* dE,
                          const RunConsts& k, hipStream_t s);
template <typename T>
hipError_t launch_drift(const Packets<T>& P, const RunConsts& k, hipStream_t s);
template <typename T>
hipError_t launch_moments(int shape, const Packets<T>& P, double* rho, double* Pm, double* e,
                          const RunConsts& k, hipStream_t s);

// fused step, one thread per packet with global atomics (any packet order); NN (nucleon
// density, precision type) selects the step with catastrophic losses (needs P.w)
template <typename T>
hipError_t launch_step_global(int shape, const Packets<T>& P, const T* E, const T* B, const T* NN, double* dM,
                              double* dE, const RunConsts& k, hipStream_t s);

// One step of the packets in their own order (Boris, no exchange deposit) that first
// writes each packet's starting state into `slab`: FP64 form [6][np] doubles (x0, x1,
// x2, u0, u1, u2); FP32 form [7][np] 4-byte words (cell, off0..2, u0..2).
template <typename T>
hipError_t launch_step_record(int shape, const Packets<T>& P, const T* E, const T* B, void* slab,
                              const RunConsts& k, hipStream_t s);

// The same step with the packets held in tile order (tile t's packets at
// [offsets[t*cells_per_tile], offsets[(t+1)*cells_per_tile]) of P, from a counting sort
// at most a few steps old): E and B of each tile plus a `halo`-cell border are staged
// in LDS, so gathers do not touch the grid.  The state is read from P and the advanced
// state written into Q at the same positions (Q may be P; a recording passes one step's
// state slab as P and the next one's as Q).  Needs step_record_tiled_fits(t, halo).
struct Tiling;
bool step_record_tiled_fits(const Tiling& t, int halo);

// The moments with the packets taken tile by tile through `order` and `offsets` (a
// counting sort of the current state), accumulated per tile plus a one-cell halo in LDS.
// Outputs as launch_moments (accumulated: zero them first).  Needs moments_tiled_fits(t).
bool moments_tiled_fits(const Tiling& t);
template <typename T>
hipError_t launch_moments_tiled(int shape, const Packets<T>& P, const int32_t* order, const int32_t* offsets,
                                const Tiling& t, double* rho, double* Pm, double* e, const RunConsts& k,
                                hipStream_t s);
template <typename T>
hipError_t launch_step_record_tiled(int shape, const Packets<T>& P, const Packets<T>& Q, const int32_t* offsets,
                                    const Tiling& t, int halo, const T* E, const T* B, const RunConsts& k,
                                    hipStream_t s);

}  // namespace rsol
