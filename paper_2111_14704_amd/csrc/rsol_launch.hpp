// Host-side launchers of the library's kernels.  Every launcher enqueues work
// on the given stream and returns the launch status; none synchronises.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rsol_particles.hpp"

namespace rsol {

constexpr int kShapeCIC = 1;
constexpr int kShapeTSC = 2;

// fields and conversions
hipError_t launch_electric_field(const double* u_gas, const double* B, double* E, int ncells,
                                 double c, hipStream_t s);
hipError_t launch_to_fp32(const double* src, float* dst, int64_t n, hipStream_t s);
hipError_t launch_positions_to_cells(const double* x, int32_t* cell, float* off, int64_t np,
                                     const RunConsts& k, hipStream_t s);
hipError_t launch_cells_to_positions(const int32_t* cell, const float* off, double* x, int64_t np,
                                     const RunConsts& k, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s);
hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t s);

// timestep inputs: out[0] = max beta (bits), out[1] = min gamma (bits), out[2] = max |B| (bits)
template <typename T>
hipError_t launch_dt_inputs(const Packets<T>& P, const double* B, int ncells,
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

// fused step, one thread per packet with global atomics (any packet order)
template <typename T>
hipError_t launch_step_global(int shape, const Packets<T>& P, const T* E, const T* B, double* dM,
                              double* dE, const RunConsts& k, hipStream_t s);

}  // namespace rsol
