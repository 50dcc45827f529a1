// Unfused kernels of the RSOL packet step: one thread per packet, any packet
// order, global FP64 atomics for every deposit.  They implement the library's
// separable phases (gather, push, deposit, drift), the CR moments, the
// timestep reductions and the field preparation, and serve as the plain GPU
// reference beside the tiled fused step.
#include <math.h>

#include "rsol_adjoint.hpp"
#include "rsol_launch.hpp"

namespace rsol {

namespace {

constexpr int kBlock = 256;

inline int grid_for(int64_t n, int block = kBlock) {
  int64_t g = (n + block - 1) / block;
  return (int)(g < 1 ? 1 : (g > 1048576 ? 1048576 : g));
}

__device__ __forceinline__ int64_t gtid() { return (int64_t)blockIdx.x * blockDim.x + threadIdx.x; }
__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }

// ---------------------------------------------------------------- fields

// E = -(u_gas/c) x B with the true c at every cell centre (Sec. 2, after Eq. (5)).
__global__ void electric_field_kernel(const double* __restrict__ u, const double* __restrict__ B,
                                      double* __restrict__ E, int nc, double inv_c) {
  for (int64_t i = gtid(); i < nc; i += gstride()) {
    const double ux = u[i], uy = u[nc + i], uz = u[2 * (int64_t)nc + i];
    const double bx = B[i], by = B[nc + i], bz = B[2 * (int64_t)nc + i];
    E[i] = -(uy * bz - uz * by) * inv_c;
    E[nc + i] = -(uz * bx - ux * bz) * inv_c;
    E[2 * (int64_t)nc + i] = -(ux * by - uy * bx) * inv_c;
  }
}

__global__ void gas_field_kernel(GasLink g, int64_t nc) {
  for (int64_t i = gtid(); i < nc; i += gstride()) gas_refresh(g, i, nc);
}

__global__ void to_fp32_kernel(const double* __restrict__ src, float* __restrict__ dst, int64_t n) {
  for (int64_t i = gtid(); i < n; i += gstride()) dst[i] = (float)src[i];
}

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, int64_t n) {
  for (int64_t i = gtid(); i < n; i += gstride()) p[i] = v;
}

__global__ void fill_f64_kernel(double* p, double v, int64_t n) {
  for (int64_t i = gtid(); i < n; i += gstride()) p[i] = v;
}

// Absolute FP64 position -> home cell + FP32 offset (the precision form's state).
__global__ void positions_to_cells_kernel(const double* __restrict__ x, int32_t* __restrict__ cell,
                                          float* __restrict__ off, int64_t np, RunConsts k) {
  const int n[3] = {k.nx, k.ny, k.nz};
  for (int64_t i = gtid(); i < np; i += gstride()) {
    int h[3];
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double s = x[d * np + i] * k.inv_dx;
      const double fl = floor(s);
      int hd = (int)fl;
      float f = (float)(s - fl);
      if (f >= 1.0f) {  // rounding to the cell edge: next cell, zero offset
        f = 0.0f;
        hd += 1;
      }
      h[d] = wrap_index(hd, n[d]);
      off[d * np + i] = f;
    }
    cell[i] = h[0] + k.nx * (h[1] + k.ny * h[2]);
  }
}

__global__ void cells_to_positions_kernel(const int32_t* __restrict__ cell, const float* __restrict__ off,
                                          double* __restrict__ x, int64_t np, RunConsts k) {
  const int nxy = k.nx * k.ny;
  for (int64_t i = gtid(); i < np; i += gstride()) {
    const int c = cell[i];
    const int iz = c / nxy;
    const int r = c - iz * nxy;
    const int iy = r / k.nx;
    const int ix = r - iy * k.nx;
    x[i] = ((double)ix + (double)off[i]) * k.dx;
    x[np + i] = ((double)iy + (double)off[np + i]) * k.dx;
    x[2 * np + i] = ((double)iz + (double)off[2 * np + i]) * k.dx;
  }
}

// ---------------------------------------------------------------- timestep inputs (Sec. 4)

__device__ __forceinline__ unsigned long long dbits(double v) { return (unsigned long long)__double_as_longlong(v); }

template <typename T>
__global__ void dt_inputs_kernel(Packets<T> P, const double* __restrict__ B, const double* __restrict__ nn, int nc,
                                 unsigned long long* out) {
  __shared__ double s_beta[kBlock], s_gamma[kBlock], s_b[kBlock], s_n[kBlock];
  double bmax = 0.0, gmin = INFINITY, bb = 0.0, nmax = 0.0;
  for (int64_t i = gtid(); i < P.np; i += gstride()) {
    const double ux = (double)P.u[i], uy = (double)P.u[P.np + i], uz = (double)P.u[2 * P.np + i];
    const double uu = ux * ux + uy * uy + uz * uz;
    const double g = sqrt(1.0 + uu);
    bmax = fmax(bmax, sqrt(uu) / g);
    gmin = fmin(gmin, g);
  }
  for (int64_t i = gtid(); i < nc; i += gstride()) {
    const double bx = B[i], by = B[nc + i], bz = B[2 * (int64_t)nc + i];
    bb = fmax(bb, sqrt(bx * bx + by * by + bz * bz));
    if (nn) nmax = fmax(nmax, fmax(nn[i], 0.0));
  }
  s_beta[threadIdx.x] = bmax;
  s_gamma[threadIdx.x] = gmin;
  s_b[threadIdx.x] = bb;
  s_n[threadIdx.x] = nmax;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s_beta[threadIdx.x] = fmax(s_beta[threadIdx.x], s_beta[threadIdx.x + w]);
      s_gamma[threadIdx.x] = fmin(s_gamma[threadIdx.x], s_gamma[threadIdx.x + w]);
      s_b[threadIdx.x] = fmax(s_b[threadIdx.x], s_b[threadIdx.x + w]);
      s_n[threadIdx.x] = fmax(s_n[threadIdx.x], s_n[threadIdx.x + w]);
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    // non-negative doubles order like their bit patterns
    atomicMax(&out[0], dbits(s_beta[0]));
    atomicMin(&out[1], dbits(s_gamma[0]));
    atomicMax(&out[2], dbits(s_b[0]));
    atomicMax(&out[3], dbits(s_n[0]));
  }
}

__global__ void dt_init_kernel(unsigned long long* out) {
  out[0] = dbits(0.0);
  out[1] = dbits(INFINITY);
  out[2] = dbits(0.0);
  out[3] = dbits(0.0);
}

// ---------------------------------------------------------------- unfused phases

template <int M, typename T>
struct Stencil {
  AxisWeights<M, T> ax, ay, az;
};

template <int M, typename T>
__device__ __forceinline__ Stencil<M, T> stencil_of(const Packets<T>& P, int64_t i, const RunConsts& k) {
  int home[3];
  T f[3];
  load_position(P, i, k, home, f);
  Stencil<M, T> s;
  s.ax = axis_weights<M, T>(home[0], f[0]);
  s.ay = axis_weights<M, T>(home[1], f[1]);
  s.az = axis_weights<M, T>(home[2], f[2]);
  return s;
}

// A4: E_p = sum_i W_i E_i, B_p = sum_i W_i B_i
template <int M, typename T>
__global__ void gather_kernel(Packets<T> P, const T* __restrict__ E, const T* __restrict__ B,
                              T* __restrict__ Ep, T* __restrict__ Bp, RunConsts k) {
  const int64_t nc = k.ncells;
  for (int64_t i = gtid(); i < P.np; i += gstride()) {
    const Stencil<M, T> s = stencil_of<M, T>(P, i, k);
    T e[3] = {0, 0, 0}, b[3] = {0, 0, 0};
    #pragma unroll
    for (int cz = 0; cz < M; ++cz) {
      const int iz = wrap_index(s.az.base + cz, k.nz);
      #pragma unroll
      for (int cy = 0; cy < M; ++cy) {
        const int iy = wrap_index(s.ay.base + cy, k.ny);
        const T wyz = s.ay.w[cy] * s.az.w[cz];
        #pragma unroll
        for (int cx = 0; cx < M; ++cx) {
          const int ix = wrap_index(s.ax.base + cx, k.nx);
          const int64_t node = ix + (int64_t)k.nx * (iy + (int64_t)k.ny * iz);
          const T w = s.ax.w[cx] * wyz;
          #pragma unroll
          for (int d = 0; d < 3; ++d) {
            e[d] += w * E[d * nc + node];
            b[d] += w * B[d * nc + node];
          }
        }
      }
    }
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      Ep[d * P.np + i] = e[d];
      Bp[d * P.np + i] = b[d];
    }
  }
}

// A5: kick u in place with pusher PUSH; payload = (du_x, du_y, du_z, dgamma)
template <typename T, int PUSH>
__global__ void push_kernel(Packets<T> P, const T* __restrict__ Ep, const T* __restrict__ Bp,
                            T* __restrict__ payload, RunConsts k) {
  const T h = (T)k.h, hb = (T)k.hb;
  const int64_t np = P.np;
  for (int64_t i = gtid(); i < np; i += gstride()) {
    const T ux = P.u[i], uy = P.u[np + i], uz = P.u[2 * np + i];
    const Kick<T> q = kick<PUSH, T>(ux, uy, uz, Ep[i], Ep[np + i], Ep[2 * np + i],
                                    Bp[i], Bp[np + i], Bp[2 * np + i], h, hb);
    P.u[i] = ux + q.dux;
    P.u[np + i] = uy + q.duy;
    P.u[2 * np + i] = uz + q.duz;
    payload[i] = q.dux;
    payload[np + i] = q.duy;
    payload[2 * np + i] = q.duz;
    payload[3 * np + i] = q.dg;
  }
}

// A6: add -(c/c_tilde) M c du W / V and -(c/c_tilde) M c^2 dgamma W / V at the current positions
template <int M, typename T>
__global__ void deposit_kernel(Packets<T> P, const T* __restrict__ payload, double* __restrict__ dM,
                               double* __restrict__ dE, RunConsts k) {
  const int64_t nc = k.ncells, np = P.np;
  for (int64_t i = gtid(); i < np; i += gstride()) {
    const Stencil<M, T> s = stencil_of<M, T>(P, i, k);
    const T qx = (T)k.pfac * payload[i], qy = (T)k.pfac * payload[np + i];
    const T qz = (T)k.pfac * payload[2 * np + i], qe = (T)k.efac * payload[3 * np + i];
    #pragma unroll
    for (int cz = 0; cz < M; ++cz) {
      const int iz = wrap_index(s.az.base + cz, k.nz);
      #pragma unroll
      for (int cy = 0; cy < M; ++cy) {
        const int iy = wrap_index(s.ay.base + cy, k.ny);
        const T wyz = s.ay.w[cy] * s.az.w[cz];
        #pragma unroll
        for (int cx = 0; cx < M; ++cx) {
          const int ix = wrap_index(s.ax.base + cx, k.nx);
          const int64_t node = ix + (int64_t)k.nx * (iy + (int64_t)k.ny * iz);
          const T w = s.ax.w[cx] * wyz;
          atomicAdd(&dM[node], (double)(w * qx));
          atomicAdd(&dM[nc + node], (double)(w * qy));
          atomicAdd(&dM[2 * nc + node], (double)(w * qz));
          if (dE) atomicAdd(&dE[node], (double)(w * qe));
        }
      }
    }
  }
}

// A7: x^{n+1} = x^n + c_tilde dt u/gamma with periodic wrap (FP64), or the
// cell + offset carry of the precision form (FP32); the position is read from P and the
// new one written into Q (the same arrays for an update in place).
template <typename T>
__device__ __forceinline__ void drift_into(const Packets<T>& P, const Packets<T>& Q, int64_t i, T ux, T uy, T uz,
                                           const RunConsts& k) {
  const int64_t np = P.np;
  bool fin;
  const T s = drift_scale<T>(ux, uy, uz, is_fp64<T>() ? (T)k.cdt : (T)k.cdt_dx, &fin);
  bool bad = !fin;
  if constexpr (is_fp64<T>()) {
    const double L[3] = {k.Lx, k.Ly, k.Lz};
    const double u3[3] = {ux, uy, uz};
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double step = s * u3[d];
      bad |= fabs(step) > k.max_step * k.dx;
      Q.x[d * np + i] = wrap_coord(P.x[d * np + i] + step, L[d]);
    }
  } else {
    const int n[3] = {k.nx, k.ny, k.nz};
    const float u3[3] = {ux, uy, uz};
    const int c = P.cell[i];
    const int nxy = k.nx * k.ny;
    int h[3];
    h[2] = c / nxy;
    const int r = c - h[2] * nxy;
    h[1] = r / k.nx;
    h[0] = r - h[1] * k.nx;
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float step = s * u3[d];
      bad |= fabsf(step) > (float)k.max_step;
      float f = P.off[d * np + i] + step;
      const float fl = floorf(f);
      int hd = h[d] + (int)fl;
      f -= fl;
      if (f >= 1.0f) {
        f = 0.0f;
        hd += 1;
      }
      h[d] = wrap_index(hd, n[d]);
      Q.off[d * np + i] = f;
    }
    Q.cell[i] = h[0] + k.nx * (h[1] + k.ny * h[2]);
  }
  if (bad) set_status(k.status, fin ? ERR_COURANT : ERR_NAN);
}

template <typename T>
__device__ __forceinline__ void drift_one(const Packets<T>& P, int64_t i, T ux, T uy, T uz, const RunConsts& k) {
  drift_into<T>(P, P, i, ux, uy, uz, k);
}

template <typename T>
__global__ void drift_kernel(Packets<T> P, RunConsts k) {
  for (int64_t i = gtid(); i < P.np; i += gstride()) {
    drift_one<T>(P, i, P.u[i], P.u[P.np + i], P.u[2 * P.np + i], k);
  }
}

// A8: rho = sum M W / V, P = sum M c u W / V, e = sum M c^2 gamma W / V
template <int M, typename T>
__global__ void moments_kernel(Packets<T> P, double* __restrict__ rho, double* __restrict__ Pm,
                               double* __restrict__ e, RunConsts k) {
  const int64_t nc = k.ncells, np = P.np;
  const double inv_v = 1.0 / (k.dx * k.dx * k.dx);
  const double m = k.mass * inv_v, mc = k.mass * k.pc * inv_v, mcc = k.mass * k.pc * k.pc * inv_v;
  for (int64_t i = gtid(); i < np; i += gstride()) {
    const Stencil<M, T> s = stencil_of<M, T>(P, i, k);
    const double ux = (double)P.u[i], uy = (double)P.u[np + i], uz = (double)P.u[2 * np + i];
    const double g = sqrt(1.0 + (ux * ux + uy * uy + uz * uz));
    const double pw = P.w ? (double)P.w[i] : 1.0;  // packet weight under losses
    #pragma unroll
    for (int cz = 0; cz < M; ++cz) {
      const int iz = wrap_index(s.az.base + cz, k.nz);
      #pragma unroll
      for (int cy = 0; cy < M; ++cy) {
        const int iy = wrap_index(s.ay.base + cy, k.ny);
        const double wyz = (double)s.ay.w[cy] * (double)s.az.w[cz];
        #pragma unroll
        for (int cx = 0; cx < M; ++cx) {
          const int ix = wrap_index(s.ax.base + cx, k.nx);
          const int64_t node = ix + (int64_t)k.nx * (iy + (int64_t)k.ny * iz);
          const double w = (double)s.ax.w[cx] * wyz * pw;
          if (rho) atomicAdd(&rho[node], w * m);
          if (Pm) {
            atomicAdd(&Pm[node], w * mc * ux);
            atomicAdd(&Pm[nc + node], w * mc * uy);
            atomicAdd(&Pm[2 * nc + node], w * mc * uz);
          }
          if (e) atomicAdd(&e[node], w * mcc * g);
        }
      }
    }
  }
}

// The same moments with the packets taken tile by tile through `order` (a counting
// sort's permutation of the current state: tile t's packets are order[offsets[t*cpt]
// .. offsets[(t+1)*cpt])).  Each workgroup accumulates one part of a tile's packets into
// its tile plus a one-cell halo in FP64 LDS and adds the region to the grid with one
// atomic per node and component.  A packet whose stencil the region does not hold (its
// sort key and its home cell disagreeing by a rounding) deposits to the grid directly.
template <int M, typename T>
__global__ void __launch_bounds__(kBlock) moments_tiled_kernel(Packets<T> P, const int32_t* __restrict__ order,
                                                               const int32_t* __restrict__ offsets, Tiling tl,
                                                               int parts, double* __restrict__ rho,
                                                               double* __restrict__ Pm, double* __restrict__ e,
                                                               RunConsts k) {
  __shared__ double Ms[5 * kAdjRegion];
  const int64_t tile = blockIdx.x / parts;
  const int part = blockIdx.x - (int)(tile * parts);
  const int ttx = (int)(tile % tl.ntx), tty = (int)((tile / tl.ntx) % tl.nty), ttz = (int)(tile / ((int64_t)tl.ntx * tl.nty));
  const int t0[3] = {ttx * tl.tx, tty * tl.ty, ttz * tl.tz};
  const int o[3] = {t0[0] - 1, t0[1] - 1, t0[2] - 1};
  const int rext[3] = {tl.tx + 2, tl.ty + 2, tl.tz + 2};
  const int rc = rext[0] * rext[1] * rext[2];
  const int pz = region_plane_pitch(rext[0], rext[1]);
  const int64_t nc = k.ncells, np = P.np;
  const double inv_v = 1.0 / (k.dx * k.dx * k.dx);
  const double m = k.mass * inv_v, mc = k.mass * k.pc * inv_v, mcc = k.mass * k.pc * k.pc * inv_v;
  for (int r = threadIdx.x; r < rc; r += blockDim.x) {
    const int s = region_index(r % rext[0], (r / rext[0]) % rext[1], r / (rext[0] * rext[1]), rext[0], pz);
    #pragma unroll
    for (int c = 0; c < 5; ++c) Ms[c * kAdjRegion + s] = 0.0;
  }
  __syncthreads();
  int64_t b0 = offsets[tile * tl.cells_per_tile], b1 = offsets[(tile + 1) * tl.cells_per_tile];
  b0 = b0 < 0 ? 0 : (b0 > np ? np : b0);
  b1 = b1 < b0 ? b0 : (b1 > np ? np : b1);
  const int64_t len = b1 - b0;
  const int64_t j0 = b0 + len * part / parts, j1 = b0 + len * (part + 1) / parts;
  const int n3[3] = {k.nx, k.ny, k.nz};
  for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
    const int64_t i = order[j];
    if (i < 0 || i >= np) continue;
    int home[3];
    T f[3];
    load_position(P, i, k, home, f);
    const double ux = (double)P.u[i], uy = (double)P.u[np + i], uz = (double)P.u[2 * np + i];
    const double g = sqrt(1.0 + (ux * ux + uy * uy + uz * uz));
    const double pw = P.w ? (double)P.w[i] : 1.0;
    bool inside = true;
    int hu[3];
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int hw = wrap_index(home[d], n3[d]);
      int delta = hw - t0[d];
      if (2 * delta >= n3[d]) delta -= n3[d];
      else if (2 * delta < -n3[d]) delta += n3[d];
      hu[d] = t0[d] + delta;
      inside &= delta + 1 >= 1 && delta + 1 <= rext[d] - 2;
    }
    const AxisWeights<M, T> ax = axis_weights<M, T>(hu[0], f[0]), ay = axis_weights<M, T>(hu[1], f[1]),
                            az = axis_weights<M, T>(hu[2], f[2]);
    #pragma unroll
    for (int cz = 0; cz < M; ++cz) {
      #pragma unroll
      for (int cy = 0; cy < M; ++cy) {
        const double wyz = (double)ay.w[cy] * (double)az.w[cz];
        #pragma unroll
        for (int cx = 0; cx < M; ++cx) {
          const double w = (double)ax.w[cx] * wyz * pw;
          const double v[5] = {w * m, w * mc * ux, w * mc * uy, w * mc * uz, w * mcc * g};
          if (inside) {
            const int s = region_index(ax.base + cx - o[0], ay.base + cy - o[1], az.base + cz - o[2], rext[0], pz);
            if (rho) atomicAdd(&Ms[s], v[0]);
            if (Pm) {
              atomicAdd(&Ms[kAdjRegion + s], v[1]);
              atomicAdd(&Ms[2 * kAdjRegion + s], v[2]);
              atomicAdd(&Ms[3 * kAdjRegion + s], v[3]);
            }
            if (e) atomicAdd(&Ms[4 * kAdjRegion + s], v[4]);
          } else {
            const int64_t node = wrap_mod(ax.base + cx, k.nx) +
                                 (int64_t)k.nx * (wrap_mod(ay.base + cy, k.ny) + (int64_t)k.ny * wrap_mod(az.base + cz, k.nz));
            if (rho) atomicAdd(&rho[node], v[0]);
            if (Pm) {
              atomicAdd(&Pm[node], v[1]);
              atomicAdd(&Pm[nc + node], v[2]);
              atomicAdd(&Pm[2 * nc + node], v[3]);
            }
            if (e) atomicAdd(&e[node], v[4]);
          }
        }
      }
    }
  }
  __syncthreads();
  for (int r = threadIdx.x; r < rc; r += blockDim.x) {
    const int ax = r % rext[0], ay = (r / rext[0]) % rext[1], az = r / (rext[0] * rext[1]);
    const int s = region_index(ax, ay, az, rext[0], pz);
    const int64_t node = wrap_mod(o[0] + ax, k.nx) +
                         (int64_t)k.nx * (wrap_mod(o[1] + ay, k.ny) + (int64_t)k.ny * wrap_mod(o[2] + az, k.nz));
    double* dst[5] = {rho, Pm, Pm ? Pm + nc : nullptr, Pm ? Pm + 2 * nc : nullptr, e};
    #pragma unroll
    for (int c = 0; c < 5; ++c) {
      const double v = Ms[c * kAdjRegion + s];
      if (dst[c] && v != 0.0) atomicAdd(&dst[c][node], v);
    }
  }
}

// Fused step with global atomics: gather at x^n, kick, exchange deposit at x^n, drift.
// LOSS: also gather the nucleon density NN, reduce the packet weight (catastrophic
// losses) and deposit the change of the weighted packet totals.  REC: write the starting
// state of each packet into the state slab `rec` (the differentiation form's recording).
template <int M, typename T, bool LOSS, int PUSH, bool REC = false>
__global__ void __launch_bounds__(kBlock) step_global_kernel(Packets<T> P, const T* __restrict__ E,
                                                             const T* __restrict__ B, const T* __restrict__ NN,
                                                             double* __restrict__ dM, double* __restrict__ dE,
                                                             RunConsts k, void* __restrict__ rec = nullptr) {
  const int64_t nc = k.ncells, np = P.np;
  const T h = (T)k.h, hb = (T)k.hb;
  for (int64_t i = gtid(); i < np; i += gstride()) {
    const Stencil<M, T> s = stencil_of<M, T>(P, i, k);
    T e[3] = {0, 0, 0}, b[3] = {0, 0, 0}, nnp = 0;
    #pragma unroll
    for (int cz = 0; cz < M; ++cz) {
      const int iz = wrap_index(s.az.base + cz, k.nz);
      #pragma unroll
      for (int cy = 0; cy < M; ++cy) {
        const int iy = wrap_index(s.ay.base + cy, k.ny);
        const T wyz = s.ay.w[cy] * s.az.w[cz];
        #pragma unroll
        for (int cx = 0; cx < M; ++cx) {
          const int ix = wrap_index(s.ax.base + cx, k.nx);
          const int64_t node = ix + (int64_t)k.nx * (iy + (int64_t)k.ny * iz);
          const T w = s.ax.w[cx] * wyz;
          #pragma unroll
          for (int d = 0; d < 3; ++d) {
            e[d] += w * E[d * nc + node];
            b[d] += w * B[d * nc + node];
          }
          if constexpr (LOSS) nnp += w * NN[node];
        }
      }
    }
    const T ux = P.u[i], uy = P.u[np + i], uz = P.u[2 * np + i];
    if constexpr (REC) store_state<T>(rec, P, i);
    const Kick<T> q = kick<PUSH, T>(ux, uy, uz, e[0], e[1], e[2], b[0], b[1], b[2], h, hb);
    const T nux = ux + q.dux, nuy = uy + q.duy, nuz = uz + q.duz;
    P.u[i] = nux;
    P.u[np + i] = nuy;
    P.u[2 * np + i] = nuz;
    T wv = T(1), wn = T(1), lost = T(0);
    if constexpr (LOSS) {
      wv = P.w[i];
      loss_step<T>(nux, nuy, nuz, nnp, (T)k.lrate, wv, &wn, &lost);
      P.w[i] = wn;
    }
    if (dM) {
      const T wl = wv * lost;
      const T qx = LOSS ? (T)k.pfac * (wn * q.dux - wl * ux) : (T)k.pfac * q.dux;
      const T qy = LOSS ? (T)k.pfac * (wn * q.duy - wl * uy) : (T)k.pfac * q.duy;
      const T qz = LOSS ? (T)k.pfac * (wn * q.duz - wl * uz) : (T)k.pfac * q.duz;
      const T qe = LOSS ? (T)k.efac * (wn * q.dg - wl * q.g0) : (T)k.efac * q.dg;
      #pragma unroll
      for (int cz = 0; cz < M; ++cz) {
        const int iz = wrap_index(s.az.base + cz, k.nz);
        #pragma unroll
        for (int cy = 0; cy < M; ++cy) {
          const int iy = wrap_index(s.ay.base + cy, k.ny);
          const T wyz = s.ay.w[cy] * s.az.w[cz];
          #pragma unroll
          for (int cx = 0; cx < M; ++cx) {
            const int ix = wrap_index(s.ax.base + cx, k.nx);
            const int64_t node = ix + (int64_t)k.nx * (iy + (int64_t)k.ny * iz);
            const T w = s.ax.w[cx] * wyz;
            atomicAdd(&dM[node], (double)(w * qx));
            atomicAdd(&dM[nc + node], (double)(w * qy));
            atomicAdd(&dM[2 * nc + node], (double)(w * qz));
            if (dE) atomicAdd(&dE[node], (double)(w * qe));
          }
        }
      }
    }
    drift_one<T>(P, i, nux, nuy, nuz, k);
  }
}

// Recording step of the differentiation form on packets held in tile order (positions
// [offsets[t*cells_per_tile], offsets[(t+1)*cells_per_tile]) belong to tile t): one
// workgroup per part of a tile stages E and B of the tile plus a `halo`-cell border in
// LDS; each packet's state is read from P and, after the gather (the weights and
// summation order of step_global_kernel, so the trajectory is the same to the bit), the
// Boris kick and the drift, written into Q at the same position (Q = P: in place; a
// recording reads one step's state slab and writes the next).  A packet whose
// stencil has left the staged region since the sort gathers from the grid instead.
template <int M, typename T>
__global__ void __launch_bounds__(kBlock) step_record_tiled_kernel(Packets<T> P, Packets<T> Q,
                                                                   const int32_t* __restrict__ offsets, Tiling tl,
                                                                   int halo, int parts, const T* __restrict__ E,
                                                                   const T* __restrict__ B, RunConsts k) {
  __shared__ T Fs[6 * kAdjRegion];
  const int64_t wg = xcd_chunk();  // neighbouring tiles on one XCD
  const int64_t tile = wg / parts;
  const int part = (int)(wg - tile * parts);
  const int ttx = (int)(tile % tl.ntx), tty = (int)((tile / tl.ntx) % tl.nty), ttz = (int)(tile / ((int64_t)tl.ntx * tl.nty));
  const int t0[3] = {ttx * tl.tx, tty * tl.ty, ttz * tl.tz};
  const int o[3] = {t0[0] - halo, t0[1] - halo, t0[2] - halo};
  const int rext[3] = {tl.tx + 2 * halo, tl.ty + 2 * halo, tl.tz + 2 * halo};
  const int rc = rext[0] * rext[1] * rext[2];
  const int pz = region_plane_pitch(rext[0], rext[1]);
  const int64_t nc = k.ncells, np = P.np;
  for (int r = threadIdx.x; r < rc; r += blockDim.x) {
    const int ax = r % rext[0], ay = (r / rext[0]) % rext[1], az = r / (rext[0] * rext[1]);
    const int64_t g = wrap_mod(o[0] + ax, k.nx) +
                      (int64_t)k.nx * (wrap_mod(o[1] + ay, k.ny) + (int64_t)k.ny * wrap_mod(o[2] + az, k.nz));
    const int s = region_index(ax, ay, az, rext[0], pz);
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      Fs[d * kAdjRegion + s] = E[d * nc + g];
      Fs[(3 + d) * kAdjRegion + s] = B[d * nc + g];
    }
  }
  __syncthreads();
  int64_t b0 = offsets[tile * tl.cells_per_tile], b1 = offsets[(tile + 1) * tl.cells_per_tile];
  b0 = b0 < 0 ? 0 : (b0 > np ? np : b0);
  b1 = b1 < b0 ? b0 : (b1 > np ? np : b1);
  const int64_t len = b1 - b0;
  const int64_t j0 = b0 + len * part / parts, j1 = b0 + len * (part + 1) / parts;
  const int n3[3] = {k.nx, k.ny, k.nz};
  const T h = (T)k.h, hb = (T)k.hb;
  for (int64_t j = j0 + threadIdx.x; j < j1; j += blockDim.x) {
    int home[3];
    T f[3];
    load_position(P, j, k, home, f);
    const T ux = P.u[j], uy = P.u[np + j], uz = P.u[2 * np + j];
    // home in the tile's unwrapped frame; the stencil spans home-1 .. home+1
    bool inside = true;
    int hu[3];
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int hw = wrap_index(home[d], n3[d]);
      int delta = hw - t0[d];
      if (2 * delta >= n3[d]) delta -= n3[d];
      else if (2 * delta < -n3[d]) delta += n3[d];
      hu[d] = t0[d] + delta;
      const int rel = delta + halo;
      inside &= rel >= 1 && rel <= rext[d] - 2;
    }
    T e[3] = {0, 0, 0}, b[3] = {0, 0, 0};
    if (inside) {
      const AxisWeights<M, T> ax = axis_weights<M, T>(hu[0], f[0]), ay = axis_weights<M, T>(hu[1], f[1]),
                              az = axis_weights<M, T>(hu[2], f[2]);
      #pragma unroll
      for (int cz = 0; cz < M; ++cz) {
        #pragma unroll
        for (int cy = 0; cy < M; ++cy) {
          const T wyz = ay.w[cy] * az.w[cz];
          #pragma unroll
          for (int cx = 0; cx < M; ++cx) {
            const int node = region_index(ax.base + cx - o[0], ay.base + cy - o[1], az.base + cz - o[2], rext[0], pz);
            const T w = ax.w[cx] * wyz;
            #pragma unroll
            for (int d = 0; d < 3; ++d) {
              e[d] += w * Fs[d * kAdjRegion + node];
              b[d] += w * Fs[(3 + d) * kAdjRegion + node];
            }
          }
        }
      }
    } else {
      const Stencil<M, T> s = stencil_of<M, T>(P, j, k);
      #pragma unroll
      for (int cz = 0; cz < M; ++cz) {
        const int iz = wrap_index(s.az.base + cz, k.nz);
        #pragma unroll
        for (int cy = 0; cy < M; ++cy) {
          const int iy = wrap_index(s.ay.base + cy, k.ny);
          const T wyz = s.ay.w[cy] * s.az.w[cz];
          #pragma unroll
          for (int cx = 0; cx < M; ++cx) {
            const int ix = wrap_index(s.ax.base + cx, k.nx);
            const int64_t node = ix + (int64_t)k.nx * (iy + (int64_t)k.ny * iz);
            const T w = s.ax.w[cx] * wyz;
            #pragma unroll
            for (int d = 0; d < 3; ++d) {
              e[d] += w * E[d * nc + node];
              b[d] += w * B[d * nc + node];
            }
          }
        }
      }
    }
    const Kick<T> q = kick<kPushBoris, T>(ux, uy, uz, e[0], e[1], e[2], b[0], b[1], b[2], h, hb);
    const T nux = ux + q.dux, nuy = uy + q.duy, nuz = uz + q.duz;
    Q.u[j] = nux;
    Q.u[np + j] = nuy;
    Q.u[2 * np + j] = nuz;
    drift_into<T>(P, Q, j, nux, nuy, nuz, k);
  }
}

}  // namespace

// ---------------------------------------------------------------- launchers

hipError_t launch_electric_field(const double* u_gas, const double* B, double* E, int ncells, double c,
                                 hipStream_t s) {
  hipLaunchKernelGGL(electric_field_kernel, dim3(grid_for(ncells)), dim3(kBlock), 0, s, u_gas, B, E, ncells,
                     1.0 / c);
  return hipGetLastError();
}

hipError_t launch_gas_field(const GasLink& g, int64_t ncells, hipStream_t s) {
  hipLaunchKernelGGL(gas_field_kernel, dim3(grid_for(ncells)), dim3(kBlock), 0, s, g, ncells);
  return hipGetLastError();
}

hipError_t launch_to_fp32(const double* src, float* dst, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(to_fp32_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, src, dst, n);
  return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill_u32_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_fill_f64(double* p, double v, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(fill_f64_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_positions_to_cells(const double* x, int32_t* cell, float* off, int64_t np,
                                     const RunConsts& k, hipStream_t s) {
  hipLaunchKernelGGL(positions_to_cells_kernel, dim3(grid_for(np)), dim3(kBlock), 0, s, x, cell, off, np, k);
  return hipGetLastError();
}

hipError_t launch_cells_to_positions(const int32_t* cell, const float* off, double* x, int64_t np,
                                     const RunConsts& k, hipStream_t s) {
  hipLaunchKernelGGL(cells_to_positions_kernel, dim3(grid_for(np)), dim3(kBlock), 0, s, cell, off, x, np, k);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_dt_inputs(const Packets<T>& P, const double* B, const double* nn, int ncells,
                            unsigned long long* out, hipStream_t s) {
  hipLaunchKernelGGL(dt_init_kernel, dim3(1), dim3(1), 0, s, out);
  const int64_t n = P.np > ncells ? P.np : ncells;
  hipLaunchKernelGGL(dt_inputs_kernel<T>, dim3(grid_for(n) > 4096 ? 4096 : grid_for(n)), dim3(kBlock), 0, s, P,
                     B, nn, ncells, out);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather(int shape, const Packets<T>& P, const T* E, const T* B, T* Ep, T* Bp,
                         const RunConsts& k, hipStream_t s) {
  if (shape == kShapeCIC)
    hipLaunchKernelGGL((gather_kernel<2, T>), dim3(grid_for(P.np)), dim3(kBlock), 0, s, P, E, B, Ep, Bp, k);
  else
    hipLaunchKernelGGL((gather_kernel<3, T>), dim3(grid_for(P.np)), dim3(kBlock), 0, s, P, E, B, Ep, Bp, k);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_push(const Packets<T>& P, const T* Ep, const T* Bp, T* payload, const RunConsts& k,
                       hipStream_t s) {
  const dim3 g(grid_for(P.np)), b(kBlock);
  if (k.pusher == kPushVay) hipLaunchKernelGGL((push_kernel<T, kPushVay>), g, b, 0, s, P, Ep, Bp, payload, k);
  else if (k.pusher == kPushHC) hipLaunchKernelGGL((push_kernel<T, kPushHC>), g, b, 0, s, P, Ep, Bp, payload, k);
  else hipLaunchKernelGGL((push_kernel<T, kPushBoris>), g, b, 0, s, P, Ep, Bp, payload, k);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_deposit(int shape, const Packets<T>& P, const T* payload, double* dM, double* dE,
                          const RunConsts& k, hipStream_t s) {
  if (shape == kShapeCIC)
    hipLaunchKernelGGL((deposit_kernel<2, T>), dim3(grid_for(P.np)), dim3(kBlock), 0, s, P, payload, dM, dE, k);
  else
    hipLaunchKernelGGL((deposit_kernel<3, T>), dim3(grid_for(P.np)), dim3(kBlock), 0, s, P, payload, dM, dE, k);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_drift(const Packets<T>& P, const RunConsts& k, hipStream_t s) {
  hipLaunchKernelGGL(drift_kernel<T>, dim3(grid_for(P.np)), dim3(kBlock), 0, s, P, k);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_moments(int shape, const Packets<T>& P, double* rho, double* Pm, double* e, const RunConsts& k,
                          hipStream_t s) {
  if (shape == kShapeCIC)
    hipLaunchKernelGGL((moments_kernel<2, T>), dim3(grid_for(P.np)), dim3(kBlock), 0, s, P, rho, Pm, e, k);
  else
    hipLaunchKernelGGL((moments_kernel<3, T>), dim3(grid_for(P.np)), dim3(kBlock), 0, s, P, rho, Pm, e, k);
  return hipGetLastError();
}

template <int M, typename T, bool L>
void step_global_variant(const Packets<T>& P, const T* E, const T* B, const T* NN, double* dM, double* dE,
                         const RunConsts& k, hipStream_t s) {
  const dim3 g(grid_for(P.np)), b(kBlock);
  if (k.pusher == kPushVay)
    hipLaunchKernelGGL((step_global_kernel<M, T, L, kPushVay>), g, b, 0, s, P, E, B, NN, dM, dE, k);
  else if (k.pusher == kPushHC)
    hipLaunchKernelGGL((step_global_kernel<M, T, L, kPushHC>), g, b, 0, s, P, E, B, NN, dM, dE, k);
  else
    hipLaunchKernelGGL((step_global_kernel<M, T, L, kPushBoris>), g, b, 0, s, P, E, B, NN, dM, dE, k);
}

template <typename T>
hipError_t launch_step_global(int shape, const Packets<T>& P, const T* E, const T* B, const T* NN, double* dM,
                              double* dE, const RunConsts& k, hipStream_t s) {
  if (NN && !P.w) return hipErrorInvalidValue;
  if (shape == kShapeCIC) {
    if (NN) step_global_variant<2, T, true>(P, E, B, NN, dM, dE, k, s);
    else step_global_variant<2, T, false>(P, E, B, NN, dM, dE, k, s);
  } else {
    if (NN) step_global_variant<3, T, true>(P, E, B, NN, dM, dE, k, s);
    else step_global_variant<3, T, false>(P, E, B, NN, dM, dE, k, s);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_step_record(int shape, const Packets<T>& P, const T* E, const T* B, void* slab, const RunConsts& k,
                              hipStream_t s) {
  if (!slab) return hipErrorInvalidValue;
  const dim3 g(grid_for(P.np)), b(kBlock);
  if (shape == kShapeCIC)
    hipLaunchKernelGGL((step_global_kernel<2, T, false, kPushBoris, true>), g, b, 0, s, P, E, B, nullptr, nullptr,
                       nullptr, k, slab);
  else
    hipLaunchKernelGGL((step_global_kernel<3, T, false, kPushBoris, true>), g, b, 0, s, P, E, B, nullptr, nullptr,
                       nullptr, k, slab);
  return hipGetLastError();
}

bool moments_tiled_fits(const Tiling& t) { return region_span(t.tx + 2, t.ty + 2, t.tz + 2) <= kAdjRegion; }

template <typename T>
hipError_t launch_moments_tiled(int shape, const Packets<T>& P, const int32_t* order, const int32_t* offsets,
                                const Tiling& t, double* rho, double* Pm, double* e, const RunConsts& k,
                                hipStream_t s) {
  if (!moments_tiled_fits(t)) return hipErrorInvalidValue;
  const int64_t ntiles = t.ntiles();
  const int64_t per_tile = (P.np + ntiles - 1) / (ntiles > 0 ? ntiles : 1);
  int parts = (int)((per_tile + 1023) / 1024);
  parts = parts < 1 ? 1 : (parts > 4 ? 4 : parts);
  const dim3 grid((unsigned)(ntiles * parts));
  if (shape == kShapeCIC)
    hipLaunchKernelGGL((moments_tiled_kernel<2, T>), grid, dim3(kBlock), 0, s, P, order, offsets, t, parts, rho, Pm,
                       e, k);
  else
    hipLaunchKernelGGL((moments_tiled_kernel<3, T>), grid, dim3(kBlock), 0, s, P, order, offsets, t, parts, rho, Pm,
                       e, k);
  return hipGetLastError();
}

bool step_record_tiled_fits(const Tiling& t, int halo) {
  return halo >= 1 && region_span(t.tx + 2 * halo, t.ty + 2 * halo, t.tz + 2 * halo) <= kAdjRegion;
}

template <typename T>
hipError_t launch_step_record_tiled(int shape, const Packets<T>& P, const Packets<T>& Q, const int32_t* offsets,
                                    const Tiling& t, int halo, const T* E, const T* B, const RunConsts& k,
                                    hipStream_t s) {
  if (!step_record_tiled_fits(t, halo)) return hipErrorInvalidValue;
  const int64_t ntiles = t.ntiles();
  const int64_t per_tile = (P.np + ntiles - 1) / (ntiles > 0 ? ntiles : 1);
  int parts = (int)((per_tile + 1023) / 1024);
  parts = parts < 1 ? 1 : (parts > 4 ? 4 : parts);
  const dim3 grid((unsigned)(ntiles * parts));
  if (shape == kShapeCIC)
    hipLaunchKernelGGL((step_record_tiled_kernel<2, T>), grid, dim3(kBlock), 0, s, P, Q, offsets, t, halo, parts, E,
                       B, k);
  else
    hipLaunchKernelGGL((step_record_tiled_kernel<3, T>), grid, dim3(kBlock), 0, s, P, Q, offsets, t, halo, parts, E,
                       B, k);
  return hipGetLastError();
}

#define RSOL_INSTANTIATE(T)                                                                                    \
  template hipError_t launch_dt_inputs<T>(const Packets<T>&, const double*, const double*, int,               \
                                          unsigned long long*, hipStream_t);                                   \
  template hipError_t launch_gather<T>(int, const Packets<T>&, const T*, const T*, T*, T*, const RunConsts&, \
                                       hipStream_t);                                                           \
  template hipError_t launch_push<T>(const Packets<T>&, const T*, const T*, T*, const RunConsts&, hipStream_t); \
  template hipError_t launch_deposit<T>(int, const Packets<T>&, const T*, double*, double*, const RunConsts&, \
                                        hipStream_t);                                                          \
  template hipError_t launch_drift<T>(const Packets<T>&, const RunConsts&, hipStream_t);                      \
  template hipError_t launch_moments<T>(int, const Packets<T>&, double*, double*, double*, const RunConsts&,  \
                                        hipStream_t);                                                          \
  template hipError_t launch_step_global<T>(int, const Packets<T>&, const T*, const T*, const T*, double*,     \
                                            double*, const RunConsts&, hipStream_t);                           \
  template hipError_t launch_step_record<T>(int, const Packets<T>&, const T*, const T*, void*, const RunConsts&, \
                                            hipStream_t);                                                      \
  template hipError_t launch_step_record_tiled<T>(int, const Packets<T>&, const Packets<T>&, const int32_t*,    \
                                                  const Tiling&, int, const T*, const T*, const RunConsts&,    \
                                                  hipStream_t);                                                \
  template hipError_t launch_moments_tiled<T>(int, const Packets<T>&, const int32_t*, const int32_t*,          \
                                              const Tiling&, double*, double*, double*, const RunConsts&,      \
                                              hipStream_t);

RSOL_INSTANTIATE(double)
RSOL_INSTANTIATE(float)

}  // namespace rsol
