// Differentiation form: forward recompute with stored states, and the hand-written
// reverse-mode adjoint of one packet step and of the CR moment deposit.
//
// Forward map of a step (Sec. 2): with W = W(x^n),
//   E_p = sum_i W_i E_i,  B_p = sum_i W_i B_i                      (gather)
//   u^{n+1} = Boris(u^n; E_p, B_p, h)                              (Eq. (11))
//   x^{n+1} = wrap(x^n + c_tilde dt u^{n+1} / gamma(u^{n+1}))      (drift)
// Its vector-Jacobian product, applied in reverse:
//   drift:  lam_u1 += c_tilde dt (lam_x / g - u1 (u1 . lam_x) / g^3), lam_x unchanged
//   kick:   (lam_u0, lam_Ep, lam_Bp) = J_Boris^T lam_u1 (derived term by term below)
//   gather: gE_i += W_i lam_Ep, gB_i += W_i lam_Bp (a scatter),
//           lam_x += sum_i grad W_i (E_i . lam_Ep + B_i . lam_Bp)
// The adjoint of the exchange deposit (a scatter) is a gather of its cotangent, and
// the adjoint of the moment deposit is a gather of the moment cotangents.
//
// These kernels run one thread per packet in the caller's packet order (no re-binning),
// so stored states and adjoint arrays stay aligned.
#include <math.h>

#include "rsol_adjoint.hpp"

namespace rsol {

namespace {

constexpr int kBlock = 256;

inline int grid_for(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  return (int)(g < 1 ? 1 : (g > 1048576 ? 1048576 : g));
}

template <typename T>
struct V3 {
  T x, y, z;
};

template <typename T>
__device__ __forceinline__ V3<T> cross(const V3<T>& a, const V3<T>& b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
template <typename T>
__device__ __forceinline__ T dot(const V3<T>& a, const V3<T>& b) {
  return a.x * b.x + a.y * b.y + a.z * b.z;
}
template <typename T>
__device__ __forceinline__ V3<T> axpy(T a, const V3<T>& x, const V3<T>& y) {
  return {a * x.x + y.x, a * x.y + y.y, a * x.z + y.z};
}

// Weights and their derivatives along the three axes at a packet.
template <int M, typename T>
struct Stencil3 {
  AxisWeights<M, T> a[3];
  T dw[3][M];  // dW/d(offset in cells)
};

template <int M, typename T>
__device__ __forceinline__ Stencil3<M, T> stencil_at(const int home[3], const T f[3]) {
  Stencil3<M, T> s;
  #pragma unroll
  for (int d = 0; d < 3; ++d) {
    s.a[d] = axis_weights<M, T>(home[d], f[d]);
    axis_weight_derivs<M, T>(home[d], f[d], s.dw[d]);
  }
  return s;
}

__device__ __forceinline__ int wrapn(int i, int n) { return i < 0 ? i + n : (i >= n ? i - n : i); }

// State of packet i in a state slab: FP64 [6][np] (x, u); FP32 [7][np] words (cell, off, u).
template <typename T>
__device__ __forceinline__ void slab_load(const void* slab, int64_t np, int64_t i, const RunConsts& k, int home[3],
                                          T f[3], double xa[3], T u[3]) {
  if constexpr (is_fp64<T>()) {
    const double* s = (const double*)slab;
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      xa[d] = s[d * np + i];
      const double q = xa[d] * k.inv_dx;
      const double fl = floor(q);
      home[d] = (int)fl;
      f[d] = q - fl;
      u[d] = s[(3 + d) * np + i];
    }
  } else {
    const int32_t* cw = (const int32_t*)slab;
    const float* fw = (const float*)slab;
    const int c = cw[i];
    const int nxy = k.nx * k.ny;
    home[2] = c / nxy;
    const int r = c - home[2] * nxy;
    home[1] = r / k.nx;
    home[0] = r - home[1] * k.nx;
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      f[d] = fw[(1 + d) * np + i];
      u[d] = fw[(4 + d) * np + i];
      xa[d] = 0.0;
    }
  }
}

template <typename T>
__device__ __forceinline__ void slab_store(void* slab, const Packets<T>& P, int64_t i) {
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

// Copy the state before the step into the slab; the step itself runs in step_global
// (launched right after on the same stream).
template <typename T>
__global__ void record_kernel(Packets<T> P, void* slab) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < P.np; i += (int64_t)gridDim.x * blockDim.x)
    slab_store<T>(slab, P, i);
}

// Reverse of one step for every packet.
template <int M, typename T>
__global__ void __launch_bounds__(kBlock) step_backward_kernel(const void* __restrict__ slab, int64_t np,
                                                               T* __restrict__ lam_x, T* __restrict__ lam_u,
                                                               const T* __restrict__ E, const T* __restrict__ B,
                                                               const double* __restrict__ lam_dM,
                                                               const double* __restrict__ lam_dE,
                                                               double* __restrict__ gE, double* __restrict__ gB,
                                                               RunConsts k) {
  const int64_t nc = k.ncells;
  const T h = (T)k.h;
  const T inv_dx = (T)k.inv_dx;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
    int home[3];
    T f[3], u0a[3];
    double xa[3];
    slab_load<T>(slab, np, i, k, home, f, xa, u0a);
    const Stencil3<M, T> st = stencil_at<M, T>(home, f);

    // ---- recompute the forward gather
    V3<T> Ep = {0, 0, 0}, Bp = {0, 0, 0};
    #pragma unroll
    for (int cz = 0; cz < M; ++cz) {
      const int iz = wrapn(st.a[2].base + cz, k.nz);
      #pragma unroll
      for (int cy = 0; cy < M; ++cy) {
        const int iy = wrapn(st.a[1].base + cy, k.ny);
        const T wyz = st.a[1].w[cy] * st.a[2].w[cz];
        #pragma unroll
        for (int cx = 0; cx < M; ++cx) {
          const int64_t node = wrapn(st.a[0].base + cx, k.nx) + (int64_t)k.nx * (iy + (int64_t)k.ny * iz);
          const T w = st.a[0].w[cx] * wyz;
          Ep.x += w * E[node];
          Ep.y += w * E[nc + node];
          Ep.z += w * E[2 * nc + node];
          Bp.x += w * B[node];
          Bp.y += w * B[nc + node];
          Bp.z += w * B[2 * nc + node];
        }
      }
    }

    // ---- recompute the Boris kick (Eq. (11)), keeping its intermediates
    const V3<T> u0 = {u0a[0], u0a[1], u0a[2]};
    const V3<T> um = axpy(h, Ep, u0);
    const T gm = sqrt(T(1) + dot(um, um));
    const T kq = h / gm;
    const V3<T> t = {kq * Bp.x, kq * Bp.y, kq * Bp.z};
    const T tt = dot(t, t);
    const T sf = T(2) / (T(1) + tt);
    const V3<T> s = {sf * t.x, sf * t.y, sf * t.z};
    const V3<T> up = [&] {
      const V3<T> c = cross(um, t);
      return V3<T>{um.x + c.x, um.y + c.y, um.z + c.z};
    }();
    const V3<T> r = cross(up, s);
    const V3<T> du = {T(2) * h * Ep.x + r.x, T(2) * h * Ep.y + r.y, T(2) * h * Ep.z + r.z};
    const V3<T> u1 = {u0.x + du.x, u0.y + du.y, u0.z + du.z};
    const T g1 = sqrt(T(1) + dot(u1, u1));

    // ---- drift adjoint: x1 = x0 + c_tilde dt u1 / g1
    V3<T> lx = {lam_x[i], lam_x[np + i], lam_x[2 * np + i]};
    V3<T> lu1 = {lam_u[i], lam_u[np + i], lam_u[2 * np + i]};
    {
      const T cd = (T)k.cdt;
      const T ig = T(1) / g1;
      const T ul = dot(u1, lx) * ig * ig * ig;
      lu1.x += cd * (lx.x * ig - u1.x * ul);
      lu1.y += cd * (lx.y * ig - u1.y * ul);
      lu1.z += cd * (lx.z * ig - u1.z * ul);
    }

    // ---- exchange-deposit adjoint (cotangent of the summed exchange, optional)
    V3<T> lu0_extra = {0, 0, 0};
    T gxw[3] = {0, 0, 0};  // d/dx of sum_i W_i (...)
    if (lam_dM) {
      V3<T> ldu = {0, 0, 0};
      T ldg = 0;
      const T pf = (T)k.pfac, ef = (T)k.efac;
      const T g0 = sqrt(T(1) + dot(u0, u0));
      const T dg = dot(du, V3<T>{u1.x + u0.x, u1.y + u0.y, u1.z + u0.z}) / (g0 + g1);
      #pragma unroll
      for (int cz = 0; cz < M; ++cz) {
        const int iz = wrapn(st.a[2].base + cz, k.nz);
        #pragma unroll
        for (int cy = 0; cy < M; ++cy) {
          const int iy = wrapn(st.a[1].base + cy, k.ny);
          #pragma unroll
          for (int cx = 0; cx < M; ++cx) {
            const int64_t node = wrapn(st.a[0].base + cx, k.nx) + (int64_t)k.nx * (iy + (int64_t)k.ny * iz);
            const T w = st.a[0].w[cx] * st.a[1].w[cy] * st.a[2].w[cz];
            const T lmx = (T)lam_dM[node], lmy = (T)lam_dM[nc + node], lmz = (T)lam_dM[2 * nc + node];
            const T le = lam_dE ? (T)lam_dE[node] : T(0);
            ldu.x += pf * w * lmx;
            ldu.y += pf * w * lmy;
            ldu.z += pf * w * lmz;
            ldg += ef * w * le;
            const T val = pf * (du.x * lmx + du.y * lmy + du.z * lmz) + ef * dg * le;
            gxw[0] += st.dw[0][cx] * st.a[1].w[cy] * st.a[2].w[cz] * val;
            gxw[1] += st.a[0].w[cx] * st.dw[1][cy] * st.a[2].w[cz] * val;
            gxw[2] += st.a[0].w[cx] * st.a[1].w[cy] * st.dw[2][cz] * val;
          }
        }
      }
      // du = u1 - u0, dgamma = gamma(u1) - gamma(u0)
      lu1.x += ldu.x + ldg * u1.x / g1;
      lu1.y += ldu.y + ldg * u1.y / g1;
      lu1.z += ldu.z + ldg * u1.z / g1;
      lu0_extra.x = -ldu.x - ldg * u0.x / g0;
      lu0_extra.y = -ldu.y - ldg * u0.y / g0;
      lu0_extra.z = -ldu.z - ldg * u0.z / g0;
    }

    // ---- Boris adjoint, in reverse order of the forward sequence
    // u1 = u+ + h E,  u+ = u- + u' x s
    V3<T> lE = {h * lu1.x, h * lu1.y, h * lu1.z};
    V3<T> lum = lu1;
    const V3<T> lup = cross(s, lu1);   // d/du' of lu1 . (u' x s)
    const V3<T> ls = cross(lu1, up);   // d/ds  of lu1 . (u' x s)
    // u' = u- + u- x t
    {
      const V3<T> c = cross(t, lup);
      lum.x += lup.x + c.x;
      lum.y += lup.y + c.y;
      lum.z += lup.z + c.z;
    }
    V3<T> lt = cross(lup, um);
    // s = sf t, sf = 2/(1 + t.t): ds/dt = sf I - sf^2 t t^T
    {
      const T tl = dot(t, ls);
      lt.x += sf * ls.x - sf * sf * tl * t.x;
      lt.y += sf * ls.y - sf * sf * tl * t.y;
      lt.z += sf * ls.z - sf * sf * tl * t.z;
    }
    // t = (h/gm) B_p
    const V3<T> lB = {kq * lt.x, kq * lt.y, kq * lt.z};
    const T lgm = -(kq / gm) * dot(Bp, lt);
    // gm = sqrt(1 + u-.u-)
    lum.x += lgm * um.x / gm;
    lum.y += lgm * um.y / gm;
    lum.z += lgm * um.z / gm;
    // u- = u0 + h E
    lE.x += h * lum.x;
    lE.y += h * lum.y;
    lE.z += h * lum.z;
    const V3<T> lu0 = {lum.x + lu0_extra.x, lum.y + lu0_extra.y, lum.z + lu0_extra.z};

    // ---- gather adjoint: scatter into gE, gB and the weight-gradient term for x
    #pragma unroll
    for (int cz = 0; cz < M; ++cz) {
      const int iz = wrapn(st.a[2].base + cz, k.nz);
      #pragma unroll
      for (int cy = 0; cy < M; ++cy) {
        const int iy = wrapn(st.a[1].base + cy, k.ny);
        #pragma unroll
        for (int cx = 0; cx < M; ++cx) {
          const int64_t node = wrapn(st.a[0].base + cx, k.nx) + (int64_t)k.nx * (iy + (int64_t)k.ny * iz);
          const T wy_wz = st.a[1].w[cy] * st.a[2].w[cz];
          const T w = st.a[0].w[cx] * wy_wz;
          atomicAdd(&gE[node], (double)(w * lE.x));
          atomicAdd(&gE[nc + node], (double)(w * lE.y));
          atomicAdd(&gE[2 * nc + node], (double)(w * lE.z));
          atomicAdd(&gB[node], (double)(w * lB.x));
          atomicAdd(&gB[nc + node], (double)(w * lB.y));
          atomicAdd(&gB[2 * nc + node], (double)(w * lB.z));
          const T val = E[node] * lE.x + E[nc + node] * lE.y + E[2 * nc + node] * lE.z + B[node] * lB.x +
                        B[nc + node] * lB.y + B[2 * nc + node] * lB.z;
          gxw[0] += st.dw[0][cx] * wy_wz * val;
          gxw[1] += st.a[0].w[cx] * st.dw[1][cy] * st.a[2].w[cz] * val;
          gxw[2] += st.a[0].w[cx] * st.a[1].w[cy] * st.dw[2][cz] * val;
        }
      }
    }
    lam_x[i] = lx.x + gxw[0] * inv_dx;
    lam_x[np + i] = lx.y + gxw[1] * inv_dx;
    lam_x[2 * np + i] = lx.z + gxw[2] * inv_dx;
    lam_u[i] = lu0.x;
    lam_u[np + i] = lu0.y;
    lam_u[2 * np + i] = lu0.z;
  }
}

// Adjoint of rsol_moments at the current state (adds into lam_x, lam_u).
template <int M, typename T>
__global__ void __launch_bounds__(kBlock) moments_backward_kernel(Packets<T> P, const double* __restrict__ lrho,
                                                                  const double* __restrict__ lP,
                                                                  const double* __restrict__ le,
                                                                  T* __restrict__ lam_x, T* __restrict__ lam_u,
                                                                  RunConsts k) {
  const int64_t nc = k.ncells, np = P.np;
  const double inv_v = 1.0 / (k.dx * k.dx * k.dx);
  const double m = k.mass * inv_v, mc = k.mass * k.c * inv_v, mcc = k.mass * k.c * k.c * inv_v;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
    int home[3];
    T f[3];
    load_position(P, i, k, home, f);
    const Stencil3<M, T> st = stencil_at<M, T>(home, f);
    const double ux = (double)P.u[i], uy = (double)P.u[np + i], uz = (double)P.u[2 * np + i];
    const double g = sqrt(1.0 + (ux * ux + uy * uy + uz * uz));
    double gu[3] = {0, 0, 0}, gx[3] = {0, 0, 0};
    double ge = 0;
    #pragma unroll
    for (int cz = 0; cz < M; ++cz) {
      const int iz = wrapn(st.a[2].base + cz, k.nz);
      #pragma unroll
      for (int cy = 0; cy < M; ++cy) {
        const int iy = wrapn(st.a[1].base + cy, k.ny);
        #pragma unroll
        for (int cx = 0; cx < M; ++cx) {
          const int64_t node = wrapn(st.a[0].base + cx, k.nx) + (int64_t)k.nx * (iy + (int64_t)k.ny * iz);
          const double wx = st.a[0].w[cx], wy = st.a[1].w[cy], wz = st.a[2].w[cz];
          const double w = wx * wy * wz;
          double val = 0;
          if (lP) {
            const double px = lP[node], py = lP[nc + node], pz = lP[2 * nc + node];
            gu[0] += mc * w * px;
            gu[1] += mc * w * py;
            gu[2] += mc * w * pz;
            val += mc * (ux * px + uy * py + uz * pz);
          }
          if (lrho) val += m * lrho[node];
          if (le) {
            ge += mcc * w * le[node];
            val += mcc * g * le[node];
          }
          gx[0] += (double)st.dw[0][cx] * wy * wz * val;
          gx[1] += wx * (double)st.dw[1][cy] * wz * val;
          gx[2] += wx * wy * (double)st.dw[2][cz] * val;
        }
      }
    }
    // d(gamma)/du = u / gamma
    gu[0] += ge * ux / g;
    gu[1] += ge * uy / g;
    gu[2] += ge * uz / g;
    lam_u[i] += (T)gu[0];
    lam_u[np + i] += (T)gu[1];
    lam_u[2 * np + i] += (T)gu[2];
    lam_x[i] += (T)(gx[0] * k.inv_dx);
    lam_x[np + i] += (T)(gx[1] * k.inv_dx);
    lam_x[2 * np + i] += (T)(gx[2] * k.inv_dx);
  }
}

}  // namespace

template <typename T>
hipError_t launch_record(const Packets<T>& P, void* slab, hipStream_t s) {
  hipLaunchKernelGGL(record_kernel<T>, dim3(grid_for(P.np)), dim3(kBlock), 0, s, P, slab);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_step_backward(int shape, const void* slab, int64_t np, T* lam_x, T* lam_u, const T* E, const T* B,
                                const double* lam_dM, const double* lam_dE, double* gE, double* gB,
                                const RunConsts& k, hipStream_t s) {
  if (shape == kShapeCIC)
    hipLaunchKernelGGL((step_backward_kernel<2, T>), dim3(grid_for(np)), dim3(kBlock), 0, s, slab, np, lam_x, lam_u, E,
                       B, lam_dM, lam_dE, gE, gB, k);
  else
    hipLaunchKernelGGL((step_backward_kernel<3, T>), dim3(grid_for(np)), dim3(kBlock), 0, s, slab, np, lam_x, lam_u, E,
                       B, lam_dM, lam_dE, gE, gB, k);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_moments_backward(int shape, const Packets<T>& P, const double* lrho, const double* lP,
                                   const double* le, T* lam_x, T* lam_u, const RunConsts& k, hipStream_t s) {
  if (shape == kShapeCIC)
    hipLaunchKernelGGL((moments_backward_kernel<2, T>), dim3(grid_for(P.np)), dim3(kBlock), 0, s, P, lrho, lP, le,
                       lam_x, lam_u, k);
  else
    hipLaunchKernelGGL((moments_backward_kernel<3, T>), dim3(grid_for(P.np)), dim3(kBlock), 0, s, P, lrho, lP, le,
                       lam_x, lam_u, k);
  return hipGetLastError();
}

#define RSOL_ADJ_INSTANTIATE(T)                                                                                 \
  template hipError_t launch_record<T>(const Packets<T>&, void*, hipStream_t);                                 \
  template hipError_t launch_step_backward<T>(int, const void*, int64_t, T*, T*, const T*, const T*,          \
                                              const double*, const double*, double*, double*, const RunConsts&, \
                                              hipStream_t);                                                    \
  template hipError_t launch_moments_backward<T>(int, const Packets<T>&, const double*, const double*,         \
                                                 const double*, T*, T*, const RunConsts&, hipStream_t);

RSOL_ADJ_INSTANTIATE(double)
RSOL_ADJ_INSTANTIATE(float)

}  // namespace rsol
