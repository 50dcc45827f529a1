// Packet-state views used by the kernels.
//
// Two layouts, both structure-of-arrays over packets:
//   FP64 form: absolute positions x[3][np] (double), momenta u[3][np] (double)
//   FP32 form: home cell index cell[np] (int32, ix + nx*(iy + ny*iz)),
//              in-cell offsets off[3][np] (float, in [0, 1) cells), momenta u[3][np] (float)
// plus a packet label id[np] (int32) that travels with every permutation.
#pragma once

#include <type_traits>

#include "rsol_device.hpp"

namespace rsol {

template <typename T>
struct Packets {
  double* x;      // FP64 form only
  int32_t* cell;  // FP32 form only
  float* off;     // FP32 form only
  T* u;
  int32_t* id;
  int64_t np;
  T* w = nullptr;  // packet weights N_j / N under catastrophic losses, NULL otherwise
};

template <typename T>
constexpr bool is_fp64() { return std::is_same<T, double>::value; }

// a / b for 0 <= a < 2^31 and b >= 1: the FP64 product with 1/b (a uniform value the
// compiler hoists out of loops) is within one of the quotient, and one comparison
// each way (remainder in 64 bits) makes it exact; cheaper than the integer division
// sequence.
__device__ __forceinline__ int div_nonneg(int a, int b) {
  const int q = (int)((double)a * (1.0 / (double)b));
  const int64_t r = (int64_t)a - (int64_t)q * b;
  return q + (r < 0 ? -1 : (r >= b ? 1 : 0));
}

// Home cell coordinates and the in-cell offset (in cells) of packet i.
template <typename T>
__device__ __forceinline__ void load_position(const Packets<T>& P, int64_t i, const RunConsts& k,
                                              int home[3], T f[3]) {
  if constexpr (is_fp64<T>()) {
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double s = P.x[d * P.np + i] * k.inv_dx;
      const double fl = floor(s);
      home[d] = (int)fl;
      f[d] = s - fl;
    }
  } else {
    const int c = P.cell[i];
    const int nxy = k.nx * k.ny;
    const int iz = div_nonneg(c, nxy);
    const int r = c - iz * nxy;
    const int iy = div_nonneg(r, k.nx);
    home[0] = r - iy * k.nx;
    home[1] = iy;
    home[2] = iz;
    #pragma unroll
    for (int d = 0; d < 3; ++d) f[d] = P.off[d * P.np + i];
  }
}

// Chunk of blockDim.x consecutive items for this workgroup: consecutive workgroups go
// to different XCDs, so when the grid is a multiple of 8 each XCD takes a contiguous
// range of chunks and the scattered accesses of its workgroups meet in its own L2.
__device__ __forceinline__ int64_t xcd_chunk() {
  const unsigned g = gridDim.x, b = blockIdx.x;
  return (g & 7u) == 0 ? (int64_t)(b & 7u) * (g >> 3) + (b >> 3) : (int64_t)b;
}

// Copy packet i's state into a state slab: FP64 [6][np] doubles (x, u); FP32 [7][np]
// 4-byte words (cell, off, u).
template <typename T>
__device__ __forceinline__ void store_state(void* slab, const Packets<T>& P, int64_t i) {
  const int64_t np = P.np;
  if constexpr (is_fp64<T>()) {
    double* s = (double*)slab;
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      s[d * np + i] = P.x[d * np + i];
      s[(3 + d) * np + i] = P.u[d * np + i];
    }
  } else {
    int32_t* cw = (int32_t*)slab;
    float* fw = (float*)slab;
    cw[i] = P.cell[i];
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      fw[(1 + d) * np + i] = P.off[d * np + i];
      fw[(4 + d) * np + i] = P.u[d * np + i];
    }
  }
}

}  // namespace rsol
