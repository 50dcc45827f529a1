// Device-side building blocks of the RSOL packet step, shared by every kernel
// of the library: run constants, the CIC/TSC assignment weights, the
// relativistic Boris kick in increment form and the periodic drift.
//
// Physics (Ji & Hopkins, arXiv:2111.14704):
//   drift      d<x>/dt = (c_tilde/c) <v> = c_tilde beta                 (Sec. 2)
//   kick       d(gamma beta)/dt = (c_tilde/c) (q/(m c)) [E + beta x B]  (Sec. 2, Eq. (11))
//   exchange   d(rho u)/dt = -sum_j (1/V_j) (c/c_tilde) d_t P_j         (Sec. 2, Eq. (12))
//   E          = -(u_gas/c) x B with the true c                         (Sec. 2, after Eq. (5))
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rsol {

// Error bits written by kernels into the library's device status word.
enum : uint32_t {
  ERR_COURANT = 1u,   // a packet moved further per step than the configured bound
  ERR_NAN = 2u,       // a non-finite momentum or position appeared
  ERR_TILE = 4u,      // a packet left the region its tile staged in LDS
};

// Per-run constants handed to every kernel by value.
struct RunConsts {
  int nx, ny, nz;
  int ncells;
  double dx, inv_dx;
  double Lx, Ly, Lz;
  double c, c_tilde, qomc, dt, mass;
  // RSOL (Eq. (11), (12)); the naive-substitution contrast mode (the momentum
  // equation of Sec. 5, item (3), with u = gamma v / c_tilde) in brackets
  double h;          // electric half kick: (c_tilde/c) (q/(m c)) dt / 2  [(c/c_tilde) (q/(m c)) dt / 2]
  double hb;         // magnetic half kick (rotation): h                  [(q/(m c)) dt / 2]
  double pc;         // speed in packet momentum M pc u, energy M pc^2 gamma: c  [c_tilde]
  double cdt;        // c_tilde dt, the drift length per unit beta
  double cdt_dx;     // c_tilde dt / dx
  double pfac;       // gas momentum per unit packet du: -(c/c_tilde) M c / V  [-M c_tilde / V]
  double efac;       // gas energy per unit packet dgamma: -(c/c_tilde) M c^2 / V  [-M c_tilde^2 / V]
  double lrate;      // catastrophic losses: (c_tilde/c) sigma c dt, the loss exponent per unit beta n_n
  int pusher;        // momentum update: kPushBoris, kPushVay or kPushHC
  double max_step;   // largest allowed |dx| per step, in cells
  uint32_t* status;  // device status word
};

__device__ __forceinline__ int wrap_index(int i, int n) {
  return i < 0 ? i + n : (i >= n ? i - n : i);
}

// Periodic index for any offset (a staged region's border can reach past one period
// of a grid only a cell or two wide).
__device__ __forceinline__ int wrap_mod(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// Axis weights from a home cell and the in-cell offset f = x/dx - home in [0, 1).
// CIC: nodes base, base+1 with base = floor(x/dx - 1/2).
// TSC: nodes home-1, home, home+1 with d = f - 1/2.
// (standard assignment functions standing in for the kernel W of Eq. (4)).
template <int M, typename T>
struct AxisWeights {
  int base;  // first node (may be -1 before wrapping)
  T w[M];
};

template <typename T>
__device__ __forceinline__ AxisWeights<2, T> cic_axis(int home, T f) {
  AxisWeights<2, T> a;
  const T half = T(0.5);
  T g;
  if (f >= half) {
    a.base = home;
    g = f - half;
  } else {
    a.base = home - 1;
    g = f + half;
  }
  a.w[0] = T(1) - g;
  a.w[1] = g;
  return a;
}

template <typename T>
__device__ __forceinline__ AxisWeights<3, T> tsc_axis(int home, T f) {
  AxisWeights<3, T> a;
  const T half = T(0.5);
  const T d = f - half;
  a.base = home - 1;
  const T l = half - d, r = half + d;
  a.w[0] = half * l * l;
  a.w[1] = T(0.75) - d * d;
  a.w[2] = half * r * r;
  return a;
}

template <int M, typename T>
__device__ __forceinline__ AxisWeights<M, T> axis_weights(int home, T f) {
  if constexpr (M == 2) {
    return cic_axis<T>(home, f);
  } else {
    return tsc_axis<T>(home, f);
  }
}

// Derivative of the axis weights with respect to the offset (per cell).
template <int M, typename T>
__device__ __forceinline__ void axis_weight_derivs(int home, T f, T dw[M]) {
  if constexpr (M == 2) {
    (void)home;
    dw[0] = T(-1);
    dw[1] = T(1);
  } else {
    (void)home;
    const T d = f - T(0.5);
    dw[0] = d - T(0.5);   // d/dd of (1/2)(1/2 - d)^2
    dw[1] = T(-2) * d;
    dw[2] = d + T(0.5);
  }
}

// Relativistic Boris kick of u = gamma*beta with electric half kick h and magnetic
// half kick hb (both (c_tilde/c) q dt/(2 m c) for Eq. (11)), written in increment
// form: du = 2 h E + u' x s equals u_new - u exactly in real arithmetic but carries
// no cancellation, and dgamma = du . (u_new + u) / (gamma_new + gamma).
template <typename T>
struct Kick {
  T dux, duy, duz, dg;
  T g0;  // gamma before the kick
};

// 1/sqrt(x) and 1/x for x >= 1 (Lorentz factors and 1 + |t|^2): the hardware
// estimate refined by Newton-Raphson steps, y <- y + y (1 - x y^2) / 2 and
// r <- r + r (1 - x r); two steps in FP64, one in FP32, each roughly doubling the
// correct bits of the estimate.  No IEEE division or square-root sequence.
template <typename T>
__device__ __forceinline__ T rsqrt_nr(T x) {
  if constexpr (sizeof(T) == 8) {
    double y = __builtin_amdgcn_rsq(x);
    double e = fma(-x * y, y, 1.0);
    y = fma(0.5 * y, e, y);
    e = fma(-x * y, y, 1.0);
    return fma(0.5 * y, e, y);
  } else {
    float y = __builtin_amdgcn_rsqf(x);
    const float e = fmaf(-x * y, y, 1.0f);
    return fmaf(0.5f * y, e, y);
  }
}

template <typename T>
__device__ __forceinline__ T rcp_nr(T x) {
  if constexpr (sizeof(T) == 8) {
    double r = __builtin_amdgcn_rcp(x);
    double e = fma(-x, r, 1.0);
    r = fma(r, e, r);
    e = fma(-x, r, 1.0);
    return fma(r, e, r);
  } else {
    float r = __builtin_amdgcn_rcpf(x);
    const float e = fmaf(-x, r, 1.0f);
    return fmaf(r, e, r);
  }
}

template <typename T>
__device__ __forceinline__ Kick<T> boris_kick(T ux, T uy, T uz, T ex, T ey, T ez,
                                              T bx, T by, T bz, T h, T hb) {
  const T hex = h * ex, hey = h * ey, hez = h * ez;
  const T mx = ux + hex, my = uy + hey, mz = uz + hez;
  const T k = hb * rsqrt_nr<T>(T(1) + (mx * mx + my * my + mz * mz));  // hb / gamma-
  const T tx = k * bx, ty = k * by, tz = k * bz;
  const T tt = tx * tx + ty * ty + tz * tz;
  const T sf = T(2) * rcp_nr<T>(T(1) + tt);
  const T sx = sf * tx, sy = sf * ty, sz = sf * tz;
  // u' = u- + u- x t
  const T px = mx + (my * tz - mz * ty);
  const T py = my + (mz * tx - mx * tz);
  const T pz = mz + (mx * ty - my * tx);
  // u+ - u- = u' x s
  const T rx = py * sz - pz * sy;
  const T ry = pz * sx - px * sz;
  const T rz = px * sy - py * sx;
  Kick<T> o;
  o.dux = (hex + hex) + rx;
  o.duy = (hey + hey) + ry;
  o.duz = (hez + hez) + rz;
  const T nx = ux + o.dux, ny = uy + o.duy, nz = uz + o.duz;
  const T q0 = T(1) + (ux * ux + uy * uy + uz * uz);
  const T q1 = T(1) + (nx * nx + ny * ny + nz * nz);
  const T g0 = q0 * rsqrt_nr<T>(q0), g1 = q1 * rsqrt_nr<T>(q1);
  o.dg = (o.dux * (nx + ux) + o.duy * (ny + uy) + o.duz * (nz + uz)) * rcp_nr<T>(g0 + g1);
  o.g0 = g0;
  return o;
}

// Momentum updates other than Boris, for the same equation du/dt = (2h/dt) E +
// (2hb/dt) beta x B: the pushers of Vay (Phys. Plasmas 15, 056701, 2008) and of Higuera
// and Cary (Phys. Plasmas 24, 052104, 2017).  Both rotate with the Lorentz factor of an
// implicit velocity average, so a packet in the force-free E x B drift keeps its
// momentum exactly.
constexpr int kPushBoris = 0;
constexpr int kPushVay = 1;
constexpr int kPushHC = 2;

// Lorentz factor of the rotation for the vector v and tau = hb B: the positive root of
// g^4 - sigma g^2 - (tau.tau + (v.tau)^2) = 0 with sigma = 1 + v.v - tau.tau.
template <typename T>
__device__ __forceinline__ T implicit_gamma(T vx, T vy, T vz, T tx, T ty, T tz) {
  const T tt = tx * tx + ty * ty + tz * tz;
  const T vt = vx * tx + vy * ty + vz * tz;
  const T sig = T(1) + (vx * vx + vy * vy + vz * vz) - tt;
  return sqrt(T(0.5) * (sig + sqrt(sig * sig + T(4) * (tt + vt * vt))));
}

// s [v + (v.t) t + v x t] with s = 1/(1 + t.t): the rotation step of both schemes.
template <typename T>
__device__ __forceinline__ void implicit_rotate(T vx, T vy, T vz, T tx, T ty, T tz, T& ox, T& oy, T& oz) {
  const T s = rcp_nr<T>(T(1) + (tx * tx + ty * ty + tz * tz));
  const T vt = vx * tx + vy * ty + vz * tz;
  ox = s * (vx + vt * tx + (vy * tz - vz * ty));
  oy = s * (vy + vt * ty + (vz * tx - vx * tz));
  oz = s * (vz + vt * tz + (vx * ty - vy * tx));
}

// du = u_new - u and dgamma = du . (u_new + u) / (gamma_new + gamma) of a finished update.
template <typename T>
__device__ __forceinline__ Kick<T> kick_from(T ux, T uy, T uz, T nx, T ny, T nz, T g0) {
  Kick<T> o;
  o.dux = nx - ux;
  o.duy = ny - uy;
  o.duz = nz - uz;
  const T q1 = T(1) + (nx * nx + ny * ny + nz * nz);
  const T g1 = q1 * rsqrt_nr<T>(q1);
  o.dg = (o.dux * (nx + ux) + o.duy * (ny + uy) + o.duz * (nz + uz)) * rcp_nr<T>(g0 + g1);
  o.g0 = g0;
  return o;
}

// Vay: u' = u + 2h E + hb (u/gamma) x B, then the implicit rotation of u' about tau = hb B.
template <typename T>
__device__ __forceinline__ Kick<T> vay_kick(T ux, T uy, T uz, T ex, T ey, T ez, T bx, T by, T bz, T h, T hb) {
  const T q0 = T(1) + (ux * ux + uy * uy + uz * uz);
  const T ig0 = rsqrt_nr<T>(q0);
  const T k = hb * ig0;
  const T px = ux + (h + h) * ex + k * (uy * bz - uz * by);
  const T py = uy + (h + h) * ey + k * (uz * bx - ux * bz);
  const T pz = uz + (h + h) * ez + k * (ux * by - uy * bx);
  const T tx0 = hb * bx, ty0 = hb * by, tz0 = hb * bz;
  const T ign = rcp_nr<T>(implicit_gamma<T>(px, py, pz, tx0, ty0, tz0));
  T nx, ny, nz;
  implicit_rotate<T>(px, py, pz, tx0 * ign, ty0 * ign, tz0 * ign, nx, ny, nz);
  return kick_from<T>(ux, uy, uz, nx, ny, nz, q0 * ig0);
}

// Higuera-Cary: u- = u + h E, implicit rotation of u- to u+, u_new = u+ + h E + u+ x t.
template <typename T>
__device__ __forceinline__ Kick<T> hc_kick(T ux, T uy, T uz, T ex, T ey, T ez, T bx, T by, T bz, T h, T hb) {
  const T q0 = T(1) + (ux * ux + uy * uy + uz * uz);
  const T g0 = q0 * rsqrt_nr<T>(q0);
  const T mx = ux + h * ex, my = uy + h * ey, mz = uz + h * ez;
  const T tx0 = hb * bx, ty0 = hb * by, tz0 = hb * bz;
  const T ign = rcp_nr<T>(implicit_gamma<T>(mx, my, mz, tx0, ty0, tz0));
  const T tx = tx0 * ign, ty = ty0 * ign, tz = tz0 * ign;
  T px, py, pz;
  implicit_rotate<T>(mx, my, mz, tx, ty, tz, px, py, pz);
  const T nx = px + h * ex + (py * tz - pz * ty);
  const T ny = py + h * ey + (pz * tx - px * tz);
  const T nz = pz + h * ez + (px * ty - py * tx);
  return kick_from<T>(ux, uy, uz, nx, ny, nz, g0);
}

// The momentum update of pusher P.
template <int P, typename T>
__device__ __forceinline__ Kick<T> kick(T ux, T uy, T uz, T ex, T ey, T ez, T bx, T by, T bz, T h, T hb) {
  if constexpr (P == kPushVay) return vay_kick<T>(ux, uy, uz, ex, ey, ez, bx, by, bz, h, hb);
  else if constexpr (P == kPushHC) return hc_kick<T>(ux, uy, uz, ex, ey, ez, bx, by, bz, h, hb);
  else return boris_kick<T>(ux, uy, uz, ex, ey, ez, bx, by, bz, h, hb);
}

// Catastrophic losses over one step (Sec. 2, collisional terms): every packet total
// decays at the reduced rate (c_tilde/c) <sigma v> n_n with <sigma v> = sigma c beta,
// beta from the new momentum u and n_n at the packet, integrated exactly over the step.
// With r = lrate beta n_n the packet keeps w exp(-r); *lost = 1 - exp(-r) is formed
// without cancellation.
template <typename T>
__device__ __forceinline__ void loss_step(T ux, T uy, T uz, T nn, T lrate, T w, T* wn, T* lost) {
  const T uu = ux * ux + uy * uy + uz * uz;
  const T beta = sqrt(uu) * rsqrt_nr<T>(T(1) + uu);
  const T r = lrate * beta * nn;
  T em1;
  if constexpr (sizeof(T) == 8) em1 = expm1(-r);
  else em1 = expm1f(-r);
  *lost = -em1;
  *wn = w + w * em1;
}

// Drift length per unit momentum, (c_tilde dt or c_tilde dt / dx) / gamma with
// gamma = sqrt(1 + |u|^2) (Sec. 2: dx/dt = c_tilde beta = c_tilde u / gamma); *ok is
// false when gamma is not finite.
template <typename T>
__device__ __forceinline__ T drift_scale(T ux, T uy, T uz, T cdt, bool* ok) {
  const T q = T(1) + (ux * ux + uy * uy + uz * uz);
  const T gi = rsqrt_nr<T>(q);
  *ok = isfinite(q) && isfinite(gi);
  return cdt * gi;
}

// Periodic wrap of an absolute coordinate into [0, L); a value that rounds to L maps
// to 0.  A step shorter than the box needs one add or subtract (exact for x in
// [-L, 2L)); longer moves take the floor form.
__device__ __forceinline__ double wrap_coord(double x, double L) {
  double y = x;
  if (y < 0.0) y += L;
  else if (y >= L) y -= L;
  if (!(y >= 0.0 && y < L)) {
    y = y - L * floor(y / L);
    if (y >= L) y -= L;
    if (y < 0.0) y = 0.0;
  }
  return y;
}

__device__ __forceinline__ void set_status(uint32_t* status, uint32_t bits) {
  atomicOr(status, bits);
}

}  // namespace rsol
