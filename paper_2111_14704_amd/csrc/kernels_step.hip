// Tiled fused packet step: one workgroup per tile of cells.
//
//  1. Stage E and B of the tile plus a halo into LDS.  The halo is the stencil
//     reach (1 cell) plus how far packets may drift between re-sorts, so every
//     packet binned to the tile at the last sort still finds its stencil here.
//  2. Each lane takes packets of the tile's segment (contiguous in HBM, laid out
//     rank-major by the sort so neighbouring lanes sit in different cells):
//     weights, gather from LDS, relativistic Boris kick of Eq. (11), exchange
//     deposit of Eq. (12) into an LDS accumulator with LDS atomics, drift.
//     A packet whose stencil left the staged region (Courant bound exceeded)
//     falls back to global loads and global atomics.
//  3. Add the LDS accumulator to the global exchange arrays with FP64 atomics.
//
// FP64 form: absolute positions, FP64 arithmetic and FP64 LDS accumulation.
// FP32 form: cell + FP32 offset, FP32 arithmetic, per-workgroup FP32 accumulation,
// FP64 global accumulation.
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "rsol_launch.hpp"
#include "rsol_step.hpp"

namespace rsol {

namespace {

// The LDS deposit accumulator is FP64 in both forms: on gfx950 the LDS FP32 atomic add
// serialises the wavefront (~190 clocks per instruction measured) while the FP64 one
// runs at ~8 clocks, so the precision form adds its FP32 products into FP64.
using Acc = double;

__device__ __forceinline__ int wrap_any(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// Local coordinate of a home cell inside a staged region of extent R starting at origin o
// (o may be negative; the region may be larger than the grid).  Returns true when the
// whole 3-point neighbourhood [lh-1, lh+1] is inside the region.
__device__ __forceinline__ bool local_coord(int home, int o, int R, int n, int& lh) {
  lh = home - o;
  if (lh < 1) lh += n * ((1 - lh + n - 1) / n);
  if (lh > R - 2) lh -= n * ((lh - (R - 2) + n - 1) / n);
  return lh >= 1 && lh <= R - 2;
}

template <int M, typename T>
__global__ void __launch_bounds__(256) step_tiled_kernel(Packets<T> src, Packets<T> dst,
                                                         const int32_t* __restrict__ offsets,
                                                         const T* __restrict__ E, const T* __restrict__ B,
                                                         double* __restrict__ dM, double* __restrict__ dE,
                                                         RunConsts k, Tiling t, Region g, int copy_id) {
  extern __shared__ __align__(16) unsigned char lds_raw[];
  const int halo = g.halo;
  const int Rx = g.rx, Ry = g.ry, Rz = g.rz;
  const int R = g.cells;  // allocated LDS cells per component (padded strides sy, sz)
  Acc* A = reinterpret_cast<Acc*>(lds_raw);  // [4][R]: momentum x,y,z, energy
  T* F = reinterpret_cast<T*>(A + 4 * R);    // [6][R]: E then B
  const bool deposit = dM != nullptr;

  // tiles are laid out so that consecutive tiles land on the same XCD (blocks are
  // dispatched round-robin over 8 XCDs): neighbouring tiles share halo fields in L2
  const int64_t ntiles = t.ntiles();
  int64_t tile = blockIdx.x;
  if ((ntiles & 7) == 0) tile = (blockIdx.x & 7) * (ntiles >> 3) + (blockIdx.x >> 3);
  const int ttx = (int)(tile % t.ntx);
  const int tty = (int)((tile / t.ntx) % t.nty);
  const int ttz = (int)(tile / ((int64_t)t.ntx * t.nty));
  const int ox = ttx * t.tx - halo, oy = tty * t.ty - halo, oz = ttz * t.tz - halo;
  const int64_t nc = k.ncells;

  const int nreg = Rx * Ry * Rz;
  for (int q = threadIdx.x; q < nreg; q += blockDim.x) {
    const int rx = q % Rx, ry = (q / Rx) % Ry, rz = q / (Rx * Ry);
    const int r = rx + g.sy * ry + g.sz * rz;
    const int64_t cell = wrap_any(ox + rx, k.nx) + (int64_t)k.nx * (wrap_any(oy + ry, k.ny) + (int64_t)k.ny * wrap_any(oz + rz, k.nz));
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      F[d * R + r] = E[d * nc + cell];
      F[(3 + d) * R + r] = B[d * nc + cell];
    }
    if (deposit) {
      #pragma unroll
      for (int d = 0; d < 4; ++d) A[d * R + r] = Acc(0);
    }
  }
  __syncthreads();

  const int64_t seg0 = offsets[tile * t.cells_per_tile];
  const int64_t seg1 = offsets[(tile + 1) * t.cells_per_tile];
  const int64_t np = src.np;
  const T h = (T)k.h, hb = (T)k.hb;
  const T pf = (T)k.pfac, ef = (T)k.efac;

  for (int64_t i = seg0 + threadIdx.x; i < seg1; i += blockDim.x) {
    // ---- position: home cell and in-cell offset
    int home[3];
    T f[3];
    double xa[3];
    if constexpr (is_fp64<T>()) {
      #pragma unroll
      for (int d = 0; d < 3; ++d) {
        xa[d] = src.x[d * np + i];
        const double s = xa[d] * k.inv_dx;
        const double fl = floor(s);
        home[d] = (int)fl;
        f[d] = s - fl;
      }
    } else {
      const int c = src.cell[i];
      const int nxy = k.nx * k.ny;
      home[2] = c / nxy;
      const int rr = c - home[2] * nxy;
      home[1] = rr / k.nx;
      home[0] = rr - home[1] * k.nx;
      #pragma unroll
      for (int d = 0; d < 3; ++d) f[d] = src.off[d * np + i];
    }
    const T ux = src.u[i], uy = src.u[np + i], uz = src.u[2 * np + i];

    const AxisWeights<M, T> ax = axis_weights<M, T>(home[0], f[0]);
    const AxisWeights<M, T> ay = axis_weights<M, T>(home[1], f[1]);
    const AxisWeights<M, T> az = axis_weights<M, T>(home[2], f[2]);
    int lx, ly, lz;
    const bool inside = local_coord(home[0], ox, Rx, k.nx, lx) & local_coord(home[1], oy, Ry, k.ny, ly) &
                        local_coord(home[2], oz, Rz, k.nz, lz);
    {
      // count packets that fall back to the global path (one atomic per wavefront)
      const unsigned long long strays = __ballot(!inside);
      if (strays) {
        const unsigned long long act = __ballot(1);
        if ((int)__lane_id() == __ffsll((long long)act) - 1) atomicAdd(k.status + 1, (uint32_t)__popcll(strays));
      }
    }

    // ---- gather E_p, B_p
    T e0 = 0, e1 = 0, e2 = 0, b0 = 0, b1 = 0, b2 = 0;
    if (inside) {
      const int bx = lx + (ax.base - home[0]), by = ly + (ay.base - home[1]), bz = lz + (az.base - home[2]);
      #pragma unroll
      for (int cz = 0; cz < M; ++cz) {
        #pragma unroll
        for (int cy = 0; cy < M; ++cy) {
          const T wyz = ay.w[cy] * az.w[cz];
          const int row = bx + g.sy * (by + cy) + g.sz * (bz + cz);
          #pragma unroll
          for (int cx = 0; cx < M; ++cx) {
            const T w = ax.w[cx] * wyz;
            const int r = row + cx;
            e0 += w * F[r];
            e1 += w * F[R + r];
            e2 += w * F[2 * R + r];
            b0 += w * F[3 * R + r];
            b1 += w * F[4 * R + r];
            b2 += w * F[5 * R + r];
          }
        }
      }
    } else {
      #pragma unroll
      for (int cz = 0; cz < M; ++cz) {
        const int iz = wrap_any(az.base + cz, k.nz);
        #pragma unroll
        for (int cy = 0; cy < M; ++cy) {
          const int iy = wrap_any(ay.base + cy, k.ny);
          const T wyz = ay.w[cy] * az.w[cz];
          #pragma unroll
          for (int cx = 0; cx < M; ++cx) {
            const int64_t node = wrap_any(ax.base + cx, k.nx) + (int64_t)k.nx * (iy + (int64_t)k.ny * iz);
            const T w = ax.w[cx] * wyz;
            e0 += w * E[node];
            e1 += w * E[nc + node];
            e2 += w * E[2 * nc + node];
            b0 += w * B[node];
            b1 += w * B[nc + node];
            b2 += w * B[2 * nc + node];
          }
        }
      }
    }

    // ---- kick (Eq. (11))
    const Kick<T> q = boris_kick<T>(ux, uy, uz, e0, e1, e2, b0, b1, b2, h, hb);
    const T nux = ux + q.dux, nuy = uy + q.duy, nuz = uz + q.duz;

    // ---- exchange deposit at x^n (Eq. (12))
    if (deposit) {
      const T qx = pf * q.dux, qy = pf * q.duy, qz = pf * q.duz, qe = ef * q.dg;
      if (inside) {
        const int bx = lx + (ax.base - home[0]), by = ly + (ay.base - home[1]), bz = lz + (az.base - home[2]);
        #pragma unroll
        for (int cz = 0; cz < M; ++cz) {
          #pragma unroll
          for (int cy = 0; cy < M; ++cy) {
            const T wyz = ay.w[cy] * az.w[cz];
            const int row = bx + g.sy * (by + cy) + g.sz * (bz + cz);
            #pragma unroll
            for (int cx = 0; cx < M; ++cx) {
              const T w = ax.w[cx] * wyz;
              const int r = row + cx;
              atomicAdd(&A[r], (Acc)(w * qx));
              atomicAdd(&A[R + r], (Acc)(w * qy));
              atomicAdd(&A[2 * R + r], (Acc)(w * qz));
              atomicAdd(&A[3 * R + r], (Acc)(w * qe));
            }
          }
        }
      } else {
        #pragma unroll
        for (int cz = 0; cz < M; ++cz) {
          const int iz = wrap_any(az.base + cz, k.nz);
          #pragma unroll
          for (int cy = 0; cy < M; ++cy) {
            const int iy = wrap_any(ay.base + cy, k.ny);
            const T wyz = ay.w[cy] * az.w[cz];
            #pragma unroll
            for (int cx = 0; cx < M; ++cx) {
              const int64_t node = wrap_any(ax.base + cx, k.nx) + (int64_t)k.nx * (iy + (int64_t)k.ny * iz);
              const T w = ax.w[cx] * wyz;
              atomicAdd(&dM[node], (double)(w * qx));
              atomicAdd(&dM[nc + node], (double)(w * qy));
              atomicAdd(&dM[2 * nc + node], (double)(w * qz));
              if (dE) atomicAdd(&dE[node], (double)(w * qe));
            }
          }
        }
      }
    }

    // ---- drift (Sec. 2: dx/dt = c_tilde beta) and store
    bool fin;
    const T s = drift_scale<T>(nux, nuy, nuz, is_fp64<T>() ? (T)k.cdt : (T)k.cdt_dx, &fin);
    bool bad = !fin;
    if constexpr (is_fp64<T>()) {
      const double L[3] = {k.Lx, k.Ly, k.Lz};
      const double un[3] = {nux, nuy, nuz};
      #pragma unroll
      for (int d = 0; d < 3; ++d) {
        const double st = s * un[d];
        bad |= fabs(st) > k.max_step * k.dx;
        dst.x[d * np + i] = wrap_coord(xa[d] + st, L[d]);
      }
    } else {
      const int n3[3] = {k.nx, k.ny, k.nz};
      const float un[3] = {nux, nuy, nuz};
      int hn[3];
      #pragma unroll
      for (int d = 0; d < 3; ++d) {
        const float st = s * un[d];
        bad |= fabsf(st) > (float)k.max_step;
        float fo = f[d] + st;
        const float fl = floorf(fo);
        int hd = home[d] + (int)fl;
        fo -= fl;
        if (fo >= 1.0f) {
          fo = 0.0f;
          hd += 1;
        }
        hn[d] = wrap_index(hd, n3[d]);
        dst.off[d * np + i] = fo;
      }
      dst.cell[i] = hn[0] + k.nx * (hn[1] + k.ny * hn[2]);
    }
    dst.u[i] = nux;
    dst.u[np + i] = nuy;
    dst.u[2 * np + i] = nuz;
    if (copy_id) dst.id[i] = src.id[i];
    if (bad) set_status(k.status, fin ? ERR_COURANT : ERR_NAN);
  }

  if (!deposit) return;
  __syncthreads();
  for (int q = threadIdx.x; q < nreg; q += blockDim.x) {
    const int rx = q % Rx, ry = (q / Rx) % Ry, rz = q / (Rx * Ry);
    const int r = rx + g.sy * ry + g.sz * rz;
    const int64_t cell = wrap_any(ox + rx, k.nx) + (int64_t)k.nx * (wrap_any(oy + ry, k.ny) + (int64_t)k.ny * wrap_any(oz + rz, k.nz));
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      const Acc v = A[d * R + r];
      if (v != Acc(0)) atomicAdd(&dM[d * nc + cell], (double)v);
    }
    const Acc v = A[3 * R + r];
    if (dE && v != Acc(0)) atomicAdd(&dE[cell], (double)v);
  }
}

}  // namespace

namespace {

// Largest number of lanes of one 32-lane half-wavefront that hit one LDS bank when a full
// rank level (one packet per tile cell, cells x-fastest) reads its home cell, for 4-byte
// (64 banks) or 8-byte (32 bank pairs) elements.  Stencil offsets shift every lane by the
// same amount, so the home pattern decides the conflicts of every access.
int bank_conflicts(int tx, int ty, int tz, int halo, int sy, int sz, int bytes) {
  const int cpt = tx * ty * tz;
  const int slots = bytes == 8 ? 32 : 64;
  int worst = 1;
  for (int base = 0; base < 64 && base < cpt; base += 32) {
    int hits[64] = {0};
    for (int l = base; l < base + 32 && l < cpt; ++l) {
      const int lx = l % tx, ly = (l / tx) % ty, lz = l / (tx * ty);
      const int idx = (lx + halo) + sy * (ly + halo) + sz * (lz + halo);
      const int b = ((idx % slots) + slots) % slots;
      if (++hits[b] > worst) worst = hits[b];
    }
  }
  return worst;
}

}  // namespace

Region make_region(const StepPlan& p) {
  Region g;
  g.halo = p.halo;
  g.rx = p.tx + 2 * p.halo;
  g.ry = p.ty + 2 * p.halo;
  g.rz = p.tz + 2 * p.halo;
  // pick the padded strides with the fewest bank conflicts (then the least padding)
  int best = 1 << 30;
  g.sy = g.rx;
  g.sz = g.rx * g.ry;
  for (int sy = g.rx; sy < g.rx + 8; ++sy) {
    for (int sz = sy * g.ry; sz < sy * g.ry + 36; ++sz) {
      const int c = bank_conflicts(p.tx, p.ty, p.tz, p.halo, sy, sz, 8) * 4 +
                    bank_conflicts(p.tx, p.ty, p.tz, p.halo, sy, sz, 4);
      const int score = c * 100000 + sz;
      if (score < best) {
        best = score;
        g.sy = sy;
        g.sz = sz;
      }
    }
  }
  g.cells = g.sz * g.rz;
  return g;
}

StepPlan plan_step(int nx, int ny, int nz, int shape, int precision, int sort_every, double courant) {
  StepPlan p;
  p.tiled = true;
  p.block = 256;
  // 64-cell tiles: one rank level of a tile fills a wavefront
  p.tx = 4;
  p.ty = 4;
  p.tz = 4;
  if (const char* env = getenv("RSOL_TILE")) {
    int a, b, c;
    if (sscanf(env, "%d,%d,%d", &a, &b, &c) == 3 && a > 0 && b > 0 && c > 0 && a * b * c <= 256) {
      p.tx = a;
      p.ty = b;
      p.tz = c;
    }
  }
  if (p.tx > nx) p.tx = nx;
  if (p.ty > ny) p.ty = ny;
  if (p.tz > nz) p.tz = nz;
  // packets move at most `courant` cells per step at the Courant timestep; between
  // re-sorts (sort_every steps) a packet can leave its tile by that much before its
  // last step in the window
  const double drift = courant * (sort_every - 1);
  p.halo = 1 + (int)ceil(drift - 1e-12);
  if (p.halo < 1) p.halo = 1;
  p.max_step = 1.0;
  (void)shape;
  (void)precision;
  return p;
}

size_t step_lds_bytes(const StepPlan& plan, int precision) {
  const Region g = make_region(plan);
  const size_t el = precision == 1 ? sizeof(float) : sizeof(double);
  return (size_t)g.cells * (4 * sizeof(double) + 6 * el);
}

template <typename T>
hipError_t launch_step_tiled(const StepPlan& plan, int shape, const Tiling& t, const Packets<T>& src,
                             const Packets<T>& dst, const int32_t* offsets, const T* E, const T* B, double* dM,
                             double* dE, const RunConsts& k, hipStream_t s) {
  const size_t lds = step_lds_bytes(plan, is_fp64<T>() ? 0 : 1);
  if (lds > 160 * 1024) return hipErrorInvalidValue;
  const int copy_id = src.id != dst.id;
  const dim3 grid((unsigned)t.ntiles()), block(256);
  const void* fn = shape == kShapeCIC ? (const void*)step_tiled_kernel<2, T> : (const void*)step_tiled_kernel<3, T>;
  if (lds > 64 * 1024) {
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  const Region g = make_region(plan);
  if (shape == kShapeCIC)
    hipLaunchKernelGGL((step_tiled_kernel<2, T>), grid, block, lds, s, src, dst, offsets, E, B, dM, dE, k, t, g,
                       copy_id);
  else
    hipLaunchKernelGGL((step_tiled_kernel<3, T>), grid, block, lds, s, src, dst, offsets, E, B, dM, dE, k, t, g,
                       copy_id);
  return hipGetLastError();
}

template hipError_t launch_step_tiled<double>(const StepPlan&, int, const Tiling&, const Packets<double>&,
                                              const Packets<double>&, const int32_t*, const double*, const double*,
                                              double*, double*, const RunConsts&, hipStream_t);
template hipError_t launch_step_tiled<float>(const StepPlan&, int, const Tiling&, const Packets<float>&,
                                             const Packets<float>&, const int32_t*, const float*, const float*,
                                             double*, double*, const RunConsts&, hipStream_t);

}  // namespace rsol
