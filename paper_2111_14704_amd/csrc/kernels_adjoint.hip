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
// The step adjoint runs either one thread per packet in the recorded order, or over
// the step's starting state counting-sorted by tile (the sorted copy carries each
// packet's index in the recorded order, through which the adjoint arrays are read and
// written), so that dL/dE and dL/dB accumulate in LDS.
#include <math.h>

#include <type_traits>

#include "rsol_adjoint.hpp"
#include "rsol_sort.hpp"

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

// Node access of the backward step.  GlobalAccess: the grid itself (wrapped indices,
// device-scope atomics for dL/dE, dL/dB).  TileAccess: a workgroup's LDS copy of the
// fields (and exchange cotangents) on its tile plus a one-cell halo, with the field
// gradients accumulated in LDS and added to the grid once per workgroup.
template <typename T>
struct GlobalAccess {
  const T* E;
  const T* B;
  const double* ldM;
  const double* ldE;
  double* gE;
  double* gB;
  int64_t nc;
  int nx, ny, nz;
  __device__ __forceinline__ int64_t node(const int base[3], int cx, int cy, int cz) const {
    return wrapn(base[0] + cx, nx) + (int64_t)nx * (wrapn(base[1] + cy, ny) + (int64_t)ny * wrapn(base[2] + cz, nz));
  }
  // E then B at node n
  __device__ __forceinline__ void fields(int64_t n, T v[6]) const {
    #pragma unroll
    for (int c = 0; c < 3; ++c) {
      v[c] = E[c * nc + n];
      v[3 + c] = B[c * nc + n];
    }
  }
  __device__ __forceinline__ bool has_ld() const { return ldM != nullptr; }
  __device__ __forceinline__ T lm(int64_t n, int c) const { return (T)ldM[c * nc + n]; }
  __device__ __forceinline__ T le(int64_t n) const { return ldE ? (T)ldE[n] : T(0); }
  // gE += w lE, gB += w lB at node n (FP64 products and sums)
  __device__ __forceinline__ void scatter(int64_t n, const double lE[3], const double lB[3], double w) const {
    #pragma unroll
    for (int c = 0; c < 3; ++c) {
      atomicAdd(&gE[c * nc + n], w * lE[c]);
      atomicAdd(&gB[c * nc + n], w * lB[c]);
    }
  }
};

template <typename T>
struct TileAccess {
  const T* F;        // [6][kAdjRegion] E then B
  const double* L;   // [4][kAdjRegion] exchange cotangents, or NULL
  double* G;         // [6][kAdjRegion] dL/dE then dL/dB accumulators
  int ox, oy, oz;    // grid coordinates of region cell 0
  int rx, pz;        // region extent along x (the row pitch) and plane pitch
  __device__ __forceinline__ int64_t node(const int base[3], int cx, int cy, int cz) const {
    return region_index(base[0] + cx - ox, base[1] + cy - oy, base[2] + cz - oz, rx, pz);
  }
  // E then B at node n (component-major: the lanes of a wave, holding packets of
  // neighbouring cells, read neighbouring words of each component)
  __device__ __forceinline__ void fields(int64_t n, T v[6]) const {
    #pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = F[c * kAdjRegion + n];
  }
  __device__ __forceinline__ bool has_ld() const { return L != nullptr; }
  __device__ __forceinline__ T lm(int64_t n, int c) const { return (T)L[c * kAdjRegion + n]; }
  __device__ __forceinline__ T le(int64_t n) const { return (T)L[3 * kAdjRegion + n]; }
  __device__ __forceinline__ void scatter(int64_t n, const double lE[3], const double lB[3], double w) const {
    #pragma unroll
    for (int c = 0; c < 3; ++c) {
      atomicAdd(&G[c * kAdjRegion + n], w * lE[c]);
      atomicAdd(&G[(3 + c) * kAdjRegion + n], w * lB[c]);
    }
  }
};

// Reverse of one step for one packet: state (home, f, u0) before the step, lam_x and
// lam_u hold dL/d(state after) on entry and dL/d(state before) on exit.
template <int M, typename T, typename A>
__device__ __forceinline__ void packet_backward(const A& acc, const int home[3], const T f[3], const T u0a[3],
                                                T lxa[3], T lua[3], const RunConsts& k) {
  const T h = (T)k.h;  // RSOL equations only: the electric and magnetic half kicks are equal
  const Stencil3<M, T> st = stencil_at<M, T>(home, f);
  const int base[3] = {st.a[0].base, st.a[1].base, st.a[2].base};

  // ---- recompute the forward gather
  V3<T> Ep = {0, 0, 0}, Bp = {0, 0, 0};
  #pragma unroll
  for (int cz = 0; cz < M; ++cz)
    #pragma unroll
    for (int cy = 0; cy < M; ++cy) {
      const T wyz = st.a[1].w[cy] * st.a[2].w[cz];
      #pragma unroll
      for (int cx = 0; cx < M; ++cx) {
        const int64_t node = acc.node(base, cx, cy, cz);
        const T w = st.a[0].w[cx] * wyz;
        T v[6];
        acc.fields(node, v);
        Ep.x += w * v[0];
        Ep.y += w * v[1];
        Ep.z += w * v[2];
        Bp.x += w * v[3];
        Bp.y += w * v[4];
        Bp.z += w * v[5];
      }
    }

  // ---- recompute the Boris kick (Eq. (11)), keeping its intermediates; Lorentz factors
  // enter through their reciprocals (hardware estimate plus Newton steps, no IEEE
  // division or square-root sequence)
  const V3<T> u0 = {u0a[0], u0a[1], u0a[2]};
  const V3<T> um = axpy(h, Ep, u0);
  const T igm = rsqrt_nr<T>(T(1) + dot(um, um));  // 1 / gamma-
  const T kq = h * igm;
  const V3<T> t = {kq * Bp.x, kq * Bp.y, kq * Bp.z};
  const T tt = dot(t, t);
  const T sf = T(2) * rcp_nr<T>(T(1) + tt);
  const V3<T> s = {sf * t.x, sf * t.y, sf * t.z};
  const V3<T> up = [&] {
    const V3<T> c = cross(um, t);
    return V3<T>{um.x + c.x, um.y + c.y, um.z + c.z};
  }();
  const V3<T> r = cross(up, s);
  const V3<T> du = {T(2) * h * Ep.x + r.x, T(2) * h * Ep.y + r.y, T(2) * h * Ep.z + r.z};
  const V3<T> u1 = {u0.x + du.x, u0.y + du.y, u0.z + du.z};
  const T g1sq = T(1) + dot(u1, u1);
  const T ig1 = rsqrt_nr<T>(g1sq);  // 1 / gamma(u1)

  // ---- drift adjoint: x1 = x0 + c_tilde dt u1 / g1
  V3<T> lx = {lxa[0], lxa[1], lxa[2]};
  V3<T> lu1 = {lua[0], lua[1], lua[2]};
  {
    const T cd = (T)k.cdt;
    const T ul = dot(u1, lx) * ig1 * ig1 * ig1;
    lu1.x += cd * (lx.x * ig1 - u1.x * ul);
    lu1.y += cd * (lx.y * ig1 - u1.y * ul);
    lu1.z += cd * (lx.z * ig1 - u1.z * ul);
  }

  // ---- exchange-deposit adjoint (cotangent of the summed exchange, optional)
  V3<T> lu0_extra = {0, 0, 0};
  T gxw[3] = {0, 0, 0};  // d/dx of sum_i W_i (...)
  if (acc.has_ld()) {
    V3<T> ldu = {0, 0, 0};
    T ldg = 0;
    const T pf = (T)k.pfac, ef = (T)k.efac;
    const T g0sq = T(1) + dot(u0, u0);
    const T ig0 = rsqrt_nr<T>(g0sq);
    // gamma(u1) - gamma(u0) = (u1 - u0) . (u1 + u0) / (gamma(u1) + gamma(u0))
    const T dg = dot(du, V3<T>{u1.x + u0.x, u1.y + u0.y, u1.z + u0.z}) * rcp_nr<T>(g0sq * ig0 + g1sq * ig1);
    #pragma unroll
    for (int cz = 0; cz < M; ++cz)
      #pragma unroll
      for (int cy = 0; cy < M; ++cy)
        #pragma unroll
        for (int cx = 0; cx < M; ++cx) {
          const int64_t node = acc.node(base, cx, cy, cz);
          const T w = st.a[0].w[cx] * st.a[1].w[cy] * st.a[2].w[cz];
          const T lmx = acc.lm(node, 0), lmy = acc.lm(node, 1), lmz = acc.lm(node, 2);
          const T le = acc.le(node);
          ldu.x += pf * w * lmx;
          ldu.y += pf * w * lmy;
          ldu.z += pf * w * lmz;
          ldg += ef * w * le;
          const T val = pf * (du.x * lmx + du.y * lmy + du.z * lmz) + ef * dg * le;
          gxw[0] += st.dw[0][cx] * st.a[1].w[cy] * st.a[2].w[cz] * val;
          gxw[1] += st.a[0].w[cx] * st.dw[1][cy] * st.a[2].w[cz] * val;
          gxw[2] += st.a[0].w[cx] * st.a[1].w[cy] * st.dw[2][cz] * val;
        }
    // du = u1 - u0, dgamma = gamma(u1) - gamma(u0)
    lu1.x += ldu.x + ldg * u1.x * ig1;
    lu1.y += ldu.y + ldg * u1.y * ig1;
    lu1.z += ldu.z + ldg * u1.z * ig1;
    lu0_extra.x = -ldu.x - ldg * u0.x * ig0;
    lu0_extra.y = -ldu.y - ldg * u0.y * ig0;
    lu0_extra.z = -ldu.z - ldg * u0.z * ig0;
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
  const T lgm = -(kq * igm) * dot(Bp, lt);
  // gamma- = sqrt(1 + u-.u-): d gamma- / d u- = u- / gamma-
  lum.x += lgm * um.x * igm;
  lum.y += lgm * um.y * igm;
  lum.z += lgm * um.z * igm;
  // u- = u0 + h E
  lE.x += h * lum.x;
  lE.y += h * lum.y;
  lE.z += h * lum.z;

  // ---- gather adjoint: scatter into gE, gB (in FP64: the cotangents are widened once
  // and each node's weight once, instead of every product) and the weight-gradient term
  // for x
  const double lEd[3] = {(double)lE.x, (double)lE.y, (double)lE.z};
  const double lBd[3] = {(double)lB.x, (double)lB.y, (double)lB.z};
  #pragma unroll
  for (int cz = 0; cz < M; ++cz)
    #pragma unroll
    for (int cy = 0; cy < M; ++cy) {
      const T wy_wz = st.a[1].w[cy] * st.a[2].w[cz];
      #pragma unroll
      for (int cx = 0; cx < M; ++cx) {
        const int64_t node = acc.node(base, cx, cy, cz);
        const T w = st.a[0].w[cx] * wy_wz;
        acc.scatter(node, lEd, lBd, (double)w);
        T v[6];
        acc.fields(node, v);
        const T val = v[0] * lE.x + v[1] * lE.y + v[2] * lE.z + v[3] * lB.x + v[4] * lB.y + v[5] * lB.z;
        gxw[0] += st.dw[0][cx] * wy_wz * val;
        gxw[1] += st.a[0].w[cx] * st.dw[1][cy] * st.a[2].w[cz] * val;
        gxw[2] += st.a[0].w[cx] * st.a[1].w[cy] * st.dw[2][cz] * val;
      }
    }
  const T inv_dx = (T)k.inv_dx;
  lxa[0] = lx.x + gxw[0] * inv_dx;
  lxa[1] = lx.y + gxw[1] * inv_dx;
  lxa[2] = lx.z + gxw[2] * inv_dx;
  lua[0] = lum.x + lu0_extra.x;
  lua[1] = lum.y + lu0_extra.y;
  lua[2] = lum.z + lu0_extra.z;
}

// Reverse of one step for every packet, in the recorded order, with device-scope
// atomics into the field gradients.
template <int M, typename T>
__global__ void __launch_bounds__(kBlock) step_backward_kernel(const void* __restrict__ slab, int64_t np,
                                                               T* __restrict__ lam_x, T* __restrict__ lam_u,
                                                               const T* __restrict__ E, const T* __restrict__ B,
                                                               const double* __restrict__ lam_dM,
                                                               const double* __restrict__ lam_dE,
                                                               double* __restrict__ gE, double* __restrict__ gB,
                                                               RunConsts k) {
  GlobalAccess<T> acc{E, B, lam_dM, lam_dE, gE, gB, (int64_t)k.ncells, k.nx, k.ny, k.nz};
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
    int home[3];
    T f[3], u0a[3];
    double xa[3];
    slab_load<T>(slab, np, i, k, home, f, xa, u0a);
    T lx[3] = {lam_x[i], lam_x[np + i], lam_x[2 * np + i]};
    T lu[3] = {lam_u[i], lam_u[np + i], lam_u[2 * np + i]};
    packet_backward<M, T>(acc, home, f, u0a, lx, lu, k);
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      lam_x[d * np + i] = lx[d];
      lam_u[d * np + i] = lu[d];
    }
  }
}

// The adjoint of a packet in the tile-ordered sweeps: one record of six values per
// packet, dL/dx then dL/du, moved with three 16-byte (FP64) or 8-byte (FP32) accesses.
template <typename T>
using Pair = typename std::conditional<is_fp64<T>(), double2, float2>::type;

template <typename T>
__device__ __forceinline__ void lam_load(const T* __restrict__ lam, int64_t i, T lx[3], T lu[3]) {
  const Pair<T>* p = reinterpret_cast<const Pair<T>*>(lam + 6 * i);
  const Pair<T> a = p[0], b = p[1], c = p[2];
  lx[0] = a.x;
  lx[1] = a.y;
  lx[2] = b.x;
  lu[0] = b.y;
  lu[1] = c.x;
  lu[2] = c.y;
}

template <typename T>
__device__ __forceinline__ void lam_store(T* __restrict__ lam, int64_t i, const T lx[3], const T lu[3]) {
  Pair<T>* p = reinterpret_cast<Pair<T>*>(lam + 6 * i);
  Pair<T> a, b, c;
  a.x = lx[0];
  a.y = lx[1];
  b.x = lx[2];
  b.y = lu[0];
  c.x = lu[1];
  c.y = lu[2];
  p[0] = a;
  p[1] = b;
  p[2] = c;
}

// Reverse of one step with the packets held in tile order: tile t's packets are entries
// [offsets[t*cells_per_tile], offsets[(t+1)*cells_per_tile]) of the slab and of the
// adjoint records lam (a counting sort of a recorded state of this step or of one up to a few steps
// earlier).  Each workgroup takes one part of one tile's packets, stages the fields of
// the tile plus a halo of `halo` cells in LDS, accumulates dL/dE, dL/dB there and adds
// the region to the grid with one atomic per node and component.  A packet whose
// stencil leaves the region (it moved further than the halo allows since the sort) is
// appended to `spill` (count in spill[parity], packet indices from spill[2]) for
// step_backward_list_kernel.  LD false: no exchange adjoint (lam_dM NULL) and no Ls
// region staged, which lets FP32 CIC run three workgroups per CU (TSC keeps the region
// and checks lam_dM at run time: without it the compiler's allocation of FP32 TSC grew
// to one wave per SIMD).
template <int M, typename T, bool LD>
__global__ void __launch_bounds__(kBlock) step_backward_tiled_kernel(Packets<T> slab,
                                                                     const int32_t* __restrict__ offsets, Tiling tl,
                                                                     int halo, int parts, int32_t* __restrict__ spill,
                                                                     int parity,
                                                                     T* __restrict__ lam, const T* __restrict__ E,
                                                                     const T* __restrict__ B,
                                                                     const double* __restrict__ lam_dM,
                                                                     const double* __restrict__ lam_dE,
                                                                     double* __restrict__ gE, double* __restrict__ gB,
                                                                     RunConsts k) {
  __shared__ T Fs[6 * kAdjRegion];
  __shared__ double Ls[LD ? 4 * kAdjRegion : 1];
  __shared__ double Gs[6 * kAdjRegion];
  const int64_t tile = blockIdx.x / parts;
  const int part = blockIdx.x - (int)(tile * parts);
  const int ttx = (int)(tile % tl.ntx), tty = (int)((tile / tl.ntx) % tl.nty), ttz = (int)(tile / ((int64_t)tl.ntx * tl.nty));
  const int t0[3] = {ttx * tl.tx, tty * tl.ty, ttz * tl.tz};
  const int ox = t0[0] - halo, oy = t0[1] - halo, oz = t0[2] - halo;
  const int rx = tl.tx + 2 * halo, ry = tl.ty + 2 * halo, rz = tl.tz + 2 * halo;
  const int rext[3] = {rx, ry, rz};
  const int rc = rx * ry * rz;
  const int pz = region_plane_pitch(rx, ry);
  const int64_t nc = k.ncells, np = slab.np;
  const bool ld = LD && lam_dM != nullptr;
  for (int r = threadIdx.x; r < rc; r += blockDim.x) {
    const int ax = r % rx, ay = (r / rx) % ry, az = r / (rx * ry);
    const int64_t g = wrap_mod(ox + ax, k.nx) + (int64_t)k.nx * (wrap_mod(oy + ay, k.ny) + (int64_t)k.ny * wrap_mod(oz + az, k.nz));
    const int s = region_index(ax, ay, az, rx, pz);
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      Fs[d * kAdjRegion + s] = E[d * nc + g];
      Fs[(3 + d) * kAdjRegion + s] = B[d * nc + g];
    }
    if constexpr (LD) {
      if (ld) {
        #pragma unroll
        for (int d = 0; d < 3; ++d) Ls[d * kAdjRegion + s] = lam_dM[d * nc + g];
        Ls[3 * kAdjRegion + s] = lam_dE ? lam_dE[g] : 0.0;
      }
    }
    #pragma unroll
    for (int d = 0; d < 6; ++d) Gs[d * kAdjRegion + s] = 0.0;
  }
  __syncthreads();
  const TileAccess<T> acc{Fs, ld ? Ls : nullptr, Gs, ox, oy, oz, rx, pz};
  // offsets come from a recorded slab: keep the range inside the arrays whatever they hold
  int64_t b0 = offsets[tile * tl.cells_per_tile], b1 = offsets[(tile + 1) * tl.cells_per_tile];
  b0 = b0 < 0 ? 0 : (b0 > np ? np : b0);
  b1 = b1 < b0 ? b0 : (b1 > np ? np : b1);
  const int64_t len = b1 - b0;
  const int64_t j0 = b0 + len * part / parts, j1 = b0 + len * (part + 1) / parts;
  const int n3[3] = {k.nx, k.ny, k.nz};
  // a packet's inputs: state before the step and the adjoint of the state after it
  struct In {
    int home[3];
    T f[3], u0[3], lx[3], lu[3];
  };
  auto load_in = [&](int64_t i, In& p) {
    load_position(slab, i, k, p.home, p.f);
    #pragma unroll
    for (int d = 0; d < 3; ++d) p.u0[d] = slab.u[d * np + i];
    lam_load(lam, i, p.lx, p.lu);
  };
  // each thread's packets in turn; without the exchange adjoint (the variant with room
  // in its registers) the next packet's inputs load while the current one is reversed
  constexpr bool kAhead = !LD;
  int64_t i = j0 + threadIdx.x;
  In cur, nxt;
  if (kAhead && i < j1) load_in(i, cur);
  for (; i < j1; i += blockDim.x) {
    if constexpr (kAhead) {
      if (i + blockDim.x < j1) load_in(i + blockDim.x, nxt);
    } else {
      load_in(i, cur);
    }
    // home in the tile's unwrapped frame; the stencil spans home-1 .. home+1
    bool inside = true;
    int hu[3];
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int hw = wrapn(cur.home[d], n3[d]);
      int delta = hw - t0[d];
      if (2 * delta >= n3[d]) delta -= n3[d];
      else if (2 * delta < -n3[d]) delta += n3[d];
      hu[d] = t0[d] + delta;
      const int rel = delta + halo;
      inside &= rel >= 1 && rel <= rext[d] - 2;
    }
    if (!inside) {
      spill[2 + atomicAdd(&spill[parity], 1)] = (int32_t)i;
    } else {
      packet_backward<M, T>(acc, hu, cur.f, cur.u0, cur.lx, cur.lu, k);
      lam_store(lam, i, cur.lx, cur.lu);
    }
    if constexpr (kAhead) cur = nxt;
  }
  __syncthreads();
  for (int r = threadIdx.x; r < rc; r += blockDim.x) {
    const int ax = r % rx, ay = (r / rx) % ry, az = r / (rx * ry);
    const int64_t g = wrap_mod(ox + ax, k.nx) + (int64_t)k.nx * (wrap_mod(oy + ay, k.ny) + (int64_t)k.ny * wrap_mod(oz + az, k.nz));
    const int s = region_index(ax, ay, az, rx, pz);
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double ge = Gs[d * kAdjRegion + s], gb = Gs[(3 + d) * kAdjRegion + s];
      if (ge != 0.0) atomicAdd(&gE[d * nc + g], ge);
      if (gb != 0.0) atomicAdd(&gB[d * nc + g], gb);
    }
  }
}

// The packets a tiled reverse step left out (spill[parity] of them, indices from
// spill[2]), with the global fields and atomics.  The other count, which the next
// (earlier) step's tiled kernel fills, is cleared here: that kernel runs after this one
// on the same stream.
template <int M, typename T>
__global__ void __launch_bounds__(kBlock) step_backward_list_kernel(Packets<T> slab, int32_t* __restrict__ spill,
                                                                    int parity, T* __restrict__ lam,
                                                                    const T* __restrict__ E,
                                                                    const T* __restrict__ B,
                                                                    const double* __restrict__ lam_dM,
                                                                    const double* __restrict__ lam_dE,
                                                                    double* __restrict__ gE, double* __restrict__ gB,
                                                                    RunConsts k) {
  const int64_t np = slab.np;
  const int n = spill[parity];
  if (blockIdx.x == 0 && threadIdx.x == 0) spill[1 - parity] = 0;
  const GlobalAccess<T> gacc{E, B, lam_dM, lam_dE, gE, gB, (int64_t)k.ncells, k.nx, k.ny, k.nz};
  for (int t = blockIdx.x * blockDim.x + threadIdx.x; t < n; t += gridDim.x * blockDim.x) {
    const int64_t i = spill[2 + t];
    int home[3];
    T f[3], u0a[3];
    load_position(slab, i, k, home, f);
    #pragma unroll
    for (int d = 0; d < 3; ++d) u0a[d] = slab.u[d * np + i];
    T lx[3], lu[3];
    lam_load(lam, i, lx, lu);
    packet_backward<M, T>(gacc, home, f, u0a, lx, lu, k);
    lam_store(lam, i, lx, lu);
  }
}

__global__ void clear_counts_kernel(int32_t* c) { c[0] = c[1] = 0; }

__global__ void iota_kernel(int32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (int32_t)i;
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
  const double m = k.mass * inv_v, mc = k.mass * k.pc * inv_v, mcc = k.mass * k.pc * k.pc * inv_v;
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

// Adjoint records between orders: dst[j] = src[idx[j]], or dst[idx[j]] = src[j] with
// scatter; idx is a permutation of 0..np-1.
template <typename T>
__global__ void permute_records_kernel(const T* __restrict__ src, T* __restrict__ dst,
                                       const int32_t* __restrict__ idx, int64_t np, bool scatter) {
  for (int64_t j = xcd_chunk() * blockDim.x + threadIdx.x; j < np; j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = idx[j];
    if (i < 0 || i >= np) continue;  // not a permutation entry (the record is left alone)
    const Pair<T>* a = reinterpret_cast<const Pair<T>*>(src + 6 * (scatter ? j : i));
    Pair<T>* b = reinterpret_cast<Pair<T>*>(dst + 6 * (scatter ? i : j));
    const Pair<T> v0 = a[0], v1 = a[1], v2 = a[2];
    b[0] = v0;
    b[1] = v1;
    b[2] = v2;
  }
}

// The caller's adjoints (lam_x [3][np], lam_u [3][np]) and records in the same order,
// one way or the other (to_rows).
template <typename T>
__global__ void records_rows_kernel(T* __restrict__ lam_x, T* __restrict__ lam_u, T* __restrict__ rec, int64_t np,
                                    bool to_rows) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < np; i += (int64_t)gridDim.x * blockDim.x) {
    T lx[3], lu[3];
    if (to_rows) {
      lam_load(rec, i, lx, lu);
      #pragma unroll
      for (int d = 0; d < 3; ++d) {
        lam_x[d * np + i] = lx[d];
        lam_u[d * np + i] = lu[d];
      }
    } else {
      #pragma unroll
      for (int d = 0; d < 3; ++d) {
        lx[d] = lam_x[d * np + i];
        lu[d] = lam_u[d * np + i];
      }
      lam_store(rec, i, lx, lu);
    }
  }
}

// Packets in tile order back to the caller's order: P[S.id[j]] = S[j] (positions and
// momenta; the caller's ids stay).  A caller order close to tile order (as rsol_sort
// leaves it) keeps each XCD's writes within a few tiles' range.
template <typename T>
__global__ void unsort_kernel(Packets<T> S, Packets<T> P) {
  const int64_t np = P.np;
  for (int64_t j = xcd_chunk() * blockDim.x + threadIdx.x; j < np; j += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = S.id[j];
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      if constexpr (is_fp64<T>()) P.x[d * np + i] = S.x[d * np + j];
      else P.off[d * np + i] = S.off[d * np + j];
      P.u[d * np + i] = S.u[d * np + j];
    }
    if constexpr (!is_fp64<T>()) P.cell[i] = S.cell[j];
  }
}

}  // namespace

template <typename T>
hipError_t launch_permute_records(const T* src, T* dst, const int32_t* idx, int64_t np, hipStream_t s) {
  if (np > 0)
    hipLaunchKernelGGL(permute_records_kernel<T>, dim3(grid_for(np)), dim3(kBlock), 0, s, src, dst, idx, np, false);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_records_rows(T* lam_x, T* lam_u, T* rec, T* tmp, const int32_t* order, int64_t np, bool to_rows,
                               hipStream_t s) {
  if (np <= 0) return hipSuccess;
  // through records in the caller's order (contiguous transposes; the permutation then
  // moves whole records)
  if (to_rows) {
    hipLaunchKernelGGL(permute_records_kernel<T>, dim3(grid_for(np)), dim3(kBlock), 0, s, rec, tmp, order, np, true);
    hipLaunchKernelGGL(records_rows_kernel<T>, dim3(grid_for(np)), dim3(kBlock), 0, s, lam_x, lam_u, tmp, np, true);
  } else {
    hipLaunchKernelGGL(records_rows_kernel<T>, dim3(grid_for(np)), dim3(kBlock), 0, s, lam_x, lam_u, tmp, np, false);
    hipLaunchKernelGGL(permute_records_kernel<T>, dim3(grid_for(np)), dim3(kBlock), 0, s, tmp, rec, order, np, false);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_unsort(const Packets<T>& S, const Packets<T>& P, hipStream_t s) {
  if (P.np > 0) hipLaunchKernelGGL(unsort_kernel<T>, dim3(grid_for(P.np)), dim3(kBlock), 0, s, S, P);
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

bool step_backward_tiled_fits(const Tiling& t, int halo) {
  return halo >= 1 && region_span(t.tx + 2 * halo, t.ty + 2 * halo, t.tz + 2 * halo) <= kAdjRegion;
}

hipError_t launch_iota(int32_t* p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(iota_kernel, dim3(grid_for(n)), dim3(kBlock), 0, s, p, n);
  return hipGetLastError();
}

hipError_t launch_spill_clear(int32_t* spill, hipStream_t s) {
  hipLaunchKernelGGL(clear_counts_kernel, dim3(1), dim3(1), 0, s, spill);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_step_backward_tiled(int shape, const Packets<T>& slab, const int32_t* offsets,
                                      const Tiling& t, int halo, int32_t* spill, int parity, T* lam, const T* E,
                                      const T* B, const double* lam_dM, const double* lam_dE, double* gE,
                                      double* gB, const RunConsts& k, hipStream_t s) {
  if (!step_backward_tiled_fits(t, halo) || (parity != 0 && parity != 1)) return hipErrorInvalidValue;
  // one workgroup per tile once the tiles alone give each of the 256 CUs two workgroups
  // (each workgroup stages and flushes its whole region, so splitting a tile costs a
  // staging and a flush per part); fewer tiles are split over up to four workgroups,
  // with at least 256 packets each, so that the chip still fills
  const int64_t ntiles = t.ntiles();
  const int64_t per_tile = (slab.np + ntiles - 1) / (ntiles > 0 ? ntiles : 1);
  constexpr int64_t kFill = 512;
  int64_t want = ntiles >= kFill ? 1 : (kFill + ntiles - 1) / (ntiles > 0 ? ntiles : 1);
  want = want > 4 ? 4 : want;
  const int64_t most = per_tile / 256 < 1 ? 1 : per_tile / 256;
  const int parts = (int)(want < most ? want : most);
  const dim3 grid((unsigned)(ntiles * parts));
  if (shape == kShapeCIC) {
    if (lam_dM)
      hipLaunchKernelGGL((step_backward_tiled_kernel<2, T, true>), grid, dim3(kBlock), 0, s, slab, offsets, t, halo,
                         parts, spill, parity, lam, E, B, lam_dM, lam_dE, gE, gB, k);
    else
      hipLaunchKernelGGL((step_backward_tiled_kernel<2, T, false>), grid, dim3(kBlock), 0, s, slab, offsets, t,
                         halo, parts, spill, parity, lam, E, B, lam_dM, lam_dE, gE, gB, k);
  } else {
    hipLaunchKernelGGL((step_backward_tiled_kernel<3, T, true>), grid, dim3(kBlock), 0, s, slab, offsets, t, halo,
                       parts, spill, parity, lam, E, B, lam_dM, lam_dE, gE, gB, k);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_step_backward_spilled(int shape, const Packets<T>& slab, int32_t* spill, int parity, T* lam,
                                        const T* E, const T* B, const double* lam_dM, const double* lam_dE,
                                        double* gE, double* gB, const RunConsts& k, hipStream_t s) {
  if (parity != 0 && parity != 1) return hipErrorInvalidValue;
  // strays are rare (packets that outran the staged halo since their block's sort): a
  // small grid keeps the launch cheap when there are none
  const dim3 lgrid((unsigned)(grid_for(slab.np) < 32 ? grid_for(slab.np) : 32));
  if (shape == kShapeCIC)
    hipLaunchKernelGGL((step_backward_list_kernel<2, T>), lgrid, dim3(kBlock), 0, s, slab, spill, parity, lam, E,
                       B, lam_dM, lam_dE, gE, gB, k);
  else
    hipLaunchKernelGGL((step_backward_list_kernel<3, T>), lgrid, dim3(kBlock), 0, s, slab, spill, parity, lam, E,
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
  template hipError_t launch_step_backward<T>(int, const void*, int64_t, T*, T*, const T*, const T*,          \
                                              const double*, const double*, double*, double*, const RunConsts&, \
                                              hipStream_t);                                                    \
  template hipError_t launch_moments_backward<T>(int, const Packets<T>&, const double*, const double*,         \
                                                 const double*, T*, T*, const RunConsts&, hipStream_t);        \
  template hipError_t launch_permute_records<T>(const T*, T*, const int32_t*, int64_t, hipStream_t);            \
  template hipError_t launch_records_rows<T>(T*, T*, T*, T*, const int32_t*, int64_t, bool, hipStream_t);       \
  template hipError_t launch_unsort<T>(const Packets<T>&, const Packets<T>&, hipStream_t);                      \
  template hipError_t launch_step_backward_tiled<T>(int, const Packets<T>&, const int32_t*,                        \
                                                    const Tiling&, int, int32_t*, int, T*, const T*, const T*,     \
                                                    const double*, const double*, double*, double*,                \
                                                    const RunConsts&, hipStream_t);                                \
  template hipError_t launch_step_backward_spilled<T>(int, const Packets<T>&, int32_t*, int, T*, const T*,         \
                                                      const T*, const double*, const double*, double*, double*,    \
                                                      const RunConsts&, hipStream_t);

RSOL_ADJ_INSTANTIATE(double)
RSOL_ADJ_INSTANTIATE(float)

}  // namespace rsol
