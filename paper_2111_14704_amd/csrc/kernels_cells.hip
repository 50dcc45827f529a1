// Cell-list fused packet step.
//
// Packets live in per-cell buckets (two ping-pong buffers), plus per-tile inboxes
// and one overflow list for the grid.  One 256-thread workgroup owns a 4x4x4 tile;
// its 64 cells map one-to-one to 64 quads (groups of 4 lanes).  A quad keeps the
// field stencil of its cell in registers: lane q < 3 holds component q of E and of
// B on the 27 nodes around the cell.  It also keeps the cell's exchange deposit in
// registers: lane q holds component q of (dM_x, dM_y, dM_z, dE) on the same 27
// nodes.  The cell's packets are taken four at a time, one per lane; the weights,
// exchange values and partial field sums of the four packets pass between the
// quad's lanes through a per-wave LDS area, so the main loop neither reads the
// field grid nor issues atomics to global memory.
//
// After its drift a packet is written straight into the bucket of its new cell
// when that cell is in the same tile (slot from an LDS counter); otherwise into
// the neighbouring tile's inbox part reserved for packets arriving from this tile
// (slot from another LDS counter; the final count is stored once, by this
// workgroup, without atomics).  The next step therefore reads every packet from
// the store of the tile it is in.  Inbox packets take a per-packet path that
// gathers from LDS-staged fields and deposits with LDS atomics; overflow packets
// (full parts, never in practice) gather from global memory and deposit with
// global atomics.  The workgroup's exchange accumulator (tile plus one-cell halo)
// is stored without atomics to a per-tile buffer that a second kernel adds into
// the grid.
//
// Physics per packet as in the other step kernels: gather at x^n, relativistic Boris
// kick of Eq. (11), exchange of Eq. (12) at x^n, drift with c_tilde beta (Sec. 2).
#include <math.h>

#include "rsol_cells.hpp"
#include "rsol_launch.hpp"
#include "rsol_sort.hpp"

namespace rsol {

namespace {

constexpr int kThreads = 256;
constexpr int kTrashSlots = 8 * kThreads;
constexpr int kRoundSlack = 2;  // quad-loop rounds beyond the tile's mean

__device__ __host__ __forceinline__ int wrapm(int i, int n) {
  i %= n;
  return i < 0 ? i + n : i;
}

// Index of a cell one step can reach, i in [-n, 2n), wrapped into [0, n) with selects
// (no integer division); anything further out (a flagged runaway step) is clamped.
__device__ __forceinline__ int wrap_near(int i, int n) {
  i = i >= n ? i - n : i;
  i = i < 0 ? i + n : i;
  return min(max(i, 0), n - 1);
}

// Per-lane strides (elements) of the quad loop's LDS exchange areas: 12 weights + 4
// exchange values, and up to 8 partial sums, padded so that the 16 quads of a wave
// (and the lanes of a wave) start on distinct 16-byte bank groups.
template <typename T>
constexpr int kPkStride = sizeof(T) == 8 ? 18 : 20;
template <typename T>
constexpr int kRsStride = 10;

// Order the wave's own LDS writes before its following LDS reads (lanes of one wave
// exchange data through LDS; no other wave touches the area).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Axis weights on the three nodes (home-1, home, home+1) for an in-cell offset f in
// [0, 1); CIC puts its two nonzero weights on (home-1, home) or (home, home+1).
template <int M, typename T>
__device__ __forceinline__ void weights3(T f, T* w) {
  const T half = T(0.5);
  if constexpr (M == 3) {
    const T d = f - half, l = half - d, r = half + d;
    w[0] = half * l * l;
    w[1] = T(0.75) - d * d;
    w[2] = half * r * r;
  } else {
    if (f >= half) {
      const T g = f - half;
      w[0] = T(0);
      w[1] = T(1) - g;
      w[2] = g;
    } else {
      const T g = f + half;
      w[0] = T(1) - g;
      w[1] = g;
      w[2] = T(0);
    }
  }
}

// One component of the field at a packet from the component's 27 node values: w[0..2]
// are the packet's x weights and w[3 + b + 3c] the products of its y and z weights
// (the quad path's CIC gather).
template <typename T>
__device__ __forceinline__ T stencil_sum(const T w[12], const T F[27]) {
  T s = T(0);
  #pragma unroll
  for (int c = 0; c < 3; ++c)
    #pragma unroll
    for (int b = 0; b < 3; ++b) {
      T t = T(0);
      #pragma unroll
      for (int a = 0; a < 3; ++a) t += w[a] * F[a + 3 * (b + 3 * c)];
      s += w[3 + b + 3 * c] * t;
    }
  return s;
}

// In place: a component's values on the 27 nodes around a cell, F[a + 3(b + 3c)], become
// the coefficients of its TSC interpolant as a polynomial in the offsets d = f - 1/2 of
// the three axes, F[i + 3(j + 3k)] multiplying dx^i dy^j dz^k.  Along one axis
// sum_a w_a(d) g_a = (g0 + 6 g1 + g2)/8 + d (g2 - g0)/2 + d^2 ((g0 + g2)/2 - g1) for the
// weights w0 = (1/2 - d)^2 / 2, w1 = 3/4 - d^2, w2 = (1/2 + d)^2 / 2.
template <typename T>
__device__ __forceinline__ void tsc_coefficients(T F[27]) {
  auto line = [&](int i0, int st) {
    const T g0 = F[i0], g1 = F[i0 + st], g2 = F[i0 + 2 * st];
    F[i0] = T(0.125) * (g0 + g2) + T(0.75) * g1;
    F[i0 + st] = T(0.5) * (g2 - g0);
    F[i0 + 2 * st] = T(0.5) * (g0 + g2) - g1;
  };
  #pragma unroll
  for (int r = 0; r < 9; ++r) line(3 * r, 1);                      // x
  #pragma unroll
  for (int r = 0; r < 9; ++r) line((r % 3) + 9 * (r / 3), 3);      // y
  #pragma unroll
  for (int r = 0; r < 9; ++r) line(r, 9);                          // z
}

// The TSC interpolant at offsets d from its coefficients (Horner along x, y, z): the
// quad path's TSC gather, 26 FMAs per component against 36 for the weighted sum, and
// only the three offsets of a packet to share across the quad.  It agrees with the
// weighted sum of gather27 to rounding, not bit for bit.
template <typename T>
__device__ __forceinline__ T tsc_poly(const T d[3], const T C[27]) {
  T q[3];
  #pragma unroll
  for (int k = 0; k < 3; ++k) {
    T r[3];
    #pragma unroll
    for (int j = 0; j < 3; ++j) {
      const int b = 3 * (j + 3 * k);
      r[j] = C[b] + d[0] * (C[b + 1] + d[0] * C[b + 2]);
    }
    q[k] = r[0] + d[1] * (r[1] + d[1] * r[2]);
  }
  return q[0] + d[2] * (q[1] + d[2] * q[2]);
}

// Interpolate NC grid components (E, B and, with losses, the nucleon density) at one
// packet from the 27 nodes around its home cell, fetch(node, comp) giving the node
// values, in the summation order of stencil_sum (x first, then y-z pairs): the
// per-packet phase's gather.
template <int NC, typename T, typename F>
__device__ __forceinline__ void gather27(const T* w, F fetch, T out[NC]) {
  #pragma unroll
  for (int d = 0; d < NC; ++d) out[d] = T(0);
  #pragma unroll
  for (int c = 0; c < 3; ++c)
    #pragma unroll
    for (int b = 0; b < 3; ++b) {
      const T wyz = w[3 + b] * w[6 + c];
      #pragma unroll
      for (int d = 0; d < NC; ++d) {
        T t = T(0);
        #pragma unroll
        for (int a = 0; a < 3; ++a) t += w[a] * fetch(a + 3 * (b + 3 * c), d);
        out[d] += wyz * t;
      }
    }
}

// Bucket slot s of local cell lc of tile t (cap a multiple of kSlotGroup): a tile's
// buckets are laid out as [slot group][cell in tile][slot in group].  A quad round
// reads one group of each of its wave's 16 cells (whole cache lines), and the four
// packets a cell files in a round mostly land in one group (one 32-byte sector in
// FP64) instead of in four rows a cache line apart.
__device__ __forceinline__ int64_t slot_index(int64_t t, int s, int lc, int cap) {
  return ((t * (cap / kSlotGroup) + s / kSlotGroup) * kCellTileCells + lc) * kSlotGroup + s % kSlotGroup;
}

// Bucket slot s of the cell with grid coordinates h.
__device__ __forceinline__ int64_t bucket_index(const int h[3], int s, int ntx, int nty, int cap) {
  const int tx = h[0] / kCellTile, ty = h[1] / kCellTile, tz = h[2] / kCellTile;
  const int64_t t = tx + (int64_t)ntx * (ty + (int64_t)nty * tz);
  const int lc = (h[0] - tx * kCellTile) + kCellTile * ((h[1] - ty * kCellTile) + kCellTile * (h[2] - tz * kCellTile));
  return slot_index(t, s, lc, cap);
}

__device__ __forceinline__ void cell_coords(int c, const RunConsts& k, int h[3]) {
  const int nxy = k.nx * k.ny;
  h[2] = c / nxy;
  const int r = c - h[2] * nxy;
  h[1] = r / k.nx;
  h[0] = r - h[1] * k.nx;
}

// Buffers of one step, current (in) and next (out).
struct StepView {
  int ntx, nty, ntz;
  int64_t ntiles;
  int cap, per_tile;
  int64_t ocap;
  int64_t ib0, ov0, tr0;
  int dcap[kDirs];
  int doff[kDirs + 1];
  SlotArrays in, out;
  const int32_t* bcnt_in;
  int32_t* bcnt_out;
  int32_t* icnt_in;   // [ntiles*kDirs] then the overflow count
  int32_t* icnt_out;
  double* halo;
};

StepView step_view(const CellLists& L) {
  StepView V;
  const int a = L.cur, b = 1 - L.cur;
  V.ntx = L.ntx;
  V.nty = L.nty;
  V.ntz = L.ntz;
  V.ntiles = L.ntiles;
  V.cap = L.cap;
  V.per_tile = L.per_tile;
  V.ocap = L.ocap;
  V.ib0 = L.ib0;
  V.ov0 = L.ov0;
  V.tr0 = L.tr0;
  for (int d = 0; d < kDirs; ++d) V.dcap[d] = L.dcap[d];
  for (int d = 0; d <= kDirs; ++d) V.doff[d] = L.doff[d];
  V.in = L.buf[a];
  V.out = L.buf[b];
  V.bcnt_in = L.bcnt[a];
  V.bcnt_out = L.bcnt[b];
  V.icnt_in = L.icnt[a];
  V.icnt_out = L.icnt[b];
  V.halo = L.halo;
  return V;
}

// Store a packet into slot j of S (FP32: its home cell into slot jc, which is a trash
// slot for buckets, where the slot implies the cell); W: with its weight wv.
template <typename T, bool W>
__device__ __forceinline__ void store_slot(const SlotArrays& S, int64_t j, int64_t jc, const double x[3],
                                           const T f[3], const T u[3], T wv, int32_t id, int32_t cell) {
  T* su = (T*)S.u;
  if constexpr (W) ((T*)S.w)[j] = wv;
  #pragma unroll
  for (int c = 0; c < 3; ++c) {
    if constexpr (is_fp64<T>()) S.x[c * S.stride + j] = x[c];
    else S.off[c * S.stride + j] = f[c];
    su[c * S.stride + j] = u[c];
  }
  S.id[j] = id;
  if constexpr (!is_fp64<T>()) S.cell[jc] = cell;
}

// Load a packet from an inbox or the overflow list (home cell not implied by the slot).
template <typename T, bool W>
__device__ __forceinline__ void load_free(const SlotArrays& S, int64_t j, const RunConsts& k, int home[3], T f[3],
                                          double xa[3], T u[3], T& wv, int32_t& id) {
  const T* su = (const T*)S.u;
  wv = W ? ((const T*)S.w)[j] : T(1);
  if constexpr (is_fp64<T>()) {
    const int n3[3] = {k.nx, k.ny, k.nz};
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      xa[d] = S.x[d * S.stride + j];
      const double s = xa[d] * k.inv_dx;
      const double fl = floor(s);
      home[d] = wrapm((int)fl, n3[d]);
      f[d] = s - fl;
    }
  } else {
    cell_coords(S.cell[j], k, home);
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      f[d] = S.off[d * S.stride + j];
      xa[d] = 0.0;
    }
  }
  #pragma unroll
  for (int d = 0; d < 3; ++d) u[d] = su[d * S.stride + j];
  id = S.id[j];
}

// Tile offset from tile tt to tile t along an axis of n tiles: -1, 0 or 1 (through
// the periodic wrap), or 2 when the tiles are not neighbours.
__device__ __forceinline__ int tile_step(int t, int tt, int n) {
  int d = t - tt;
  if (n > 2) {
    if (d == n - 1) d = -1;
    else if (d == 1 - n) d = 1;
  }
  return (d < -1 || d > 1) ? 2 : d;
}

// Slot (in the next buffer) for a packet of this workgroup's tile whose new (wrapped)
// home cell is h: the bucket of h when h is in this tile and the bucket has room,
// else the part of h's tile inbox reserved for packets from this tile.  Returns -1
// when neither has room or h's tile is not a neighbour (the packet then needs an
// overflow slot).  *bucket tells whether the slot is a bucket slot.
__device__ __forceinline__ int64_t place(const StepView& V, int ttx, int tty, int ttz, int* cntB, int* cntD,
                                         const int* sDcap, const int* sDoff, const int h[3], bool* bucket) {
  // h is a wrapped cell index (non-negative): tile and cell in tile by shifts and masks
  const int tx = (int)((unsigned)h[0] / kCellTile), ty = (int)((unsigned)h[1] / kCellTile),
            tz = (int)((unsigned)h[2] / kCellTile);
  const int sx = tile_step(tx, ttx, V.ntx), sy = tile_step(ty, tty, V.nty), sz = tile_step(tz, ttz, V.ntz);
  *bucket = false;
  if (sx > 1 || sy > 1 || sz > 1) return -1;
  const int dir = (sx + 1) + 3 * ((sy + 1) + 3 * (sz + 1));
  if (dir == kSelfDir) {
    const int local = (int)((unsigned)h[0] % kCellTile) +
                      kCellTile * ((int)((unsigned)h[1] % kCellTile) + kCellTile * (int)((unsigned)h[2] % kCellTile));
    const int slot = atomicAdd(&cntB[local], 1);
    if (slot < V.cap) {
      *bucket = true;
      const int64_t t = tx + (int64_t)V.ntx * (ty + (int64_t)V.nty * tz);
      return slot_index(t, slot, local, V.cap);
    }
  }
  const int s = atomicAdd(&cntD[dir], 1);
  if (s < sDcap[dir]) {
    const int64_t t = tx + (int64_t)V.ntx * (ty + (int64_t)V.nty * tz);
    return V.ib0 + t * V.per_tile + sDoff[dir] + s;
  }
  return -1;
}

// Slot in the next overflow list (global counter), or the trash slot and ERR_TILE
// when that is full too (unreachable: the list holds every packet).
__device__ __forceinline__ int64_t place_overflow(const StepView& V, int64_t trash, uint32_t& err) {
  const int s = atomicAdd(V.icnt_out + V.ntiles * kDirs, 1);
  if ((int64_t)s < V.ocap) return V.ov0 + s;
  err |= ERR_TILE;
  return trash;
}

// Drift (Sec. 2: dx/dt = c_tilde beta) of one packet with home cell `home`, offset f
// (cells) and FP64 position xa; returns the new home h, position xn (FP64) and
// offset fn (FP32), and error bits.
template <typename T>
__device__ __forceinline__ uint32_t drift3(const RunConsts& k, const int home[3], const T f[3], const double xa[3],
                                           const T un[3], int h[3], double xn[3], T fn[3]) {
  bool fin;
  const T s = drift_scale<T>(un[0], un[1], un[2], is_fp64<T>() ? (T)k.cdt : (T)k.cdt_dx, &fin);
  bool bad = !fin;
  const int n3[3] = {k.nx, k.ny, k.nz};
  if constexpr (is_fp64<T>()) {
    const double L3[3] = {k.Lx, k.Ly, k.Lz};
    // periodic wrap with selects (a step moves less than one box length); one rare
    // branch takes what is still outside [0, L) (a flagged runaway or non-finite step)
    bool out = false;
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double st = s * un[d];
      bad |= fabs(st) > k.max_step * k.dx;
      double y = xa[d] + st;
      y = y < 0.0 ? y + L3[d] : y;
      y = y >= L3[d] ? y - L3[d] : y;
      out |= !(y >= 0.0 && y < L3[d]);
      xn[d] = y;
      fn[d] = 0;
    }
    if (out) {
      #pragma unroll
      for (int d = 0; d < 3; ++d) xn[d] = wrap_coord(xn[d], L3[d]);
    }
    #pragma unroll
    for (int d = 0; d < 3; ++d) h[d] = wrap_near((int)floor(xn[d] * k.inv_dx), n3[d]);
  } else {
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
      h[d] = wrap_near(hd, n3[d]);
      fn[d] = fo;
      xn[d] = 0.0;
    }
  }
  if (!bad) return 0u;
  return fin ? (uint32_t)ERR_COURANT : (uint32_t)ERR_NAN;
}

// LOSS: catastrophic losses.  The tile stages the nucleon density NN as a seventh
// field, the quad's lane 3 (idle in the field gather otherwise) gathers it, and the
// packet weight travels with the packet through the slot stores.  PUSH: the momentum
// update (Boris, Vay or Higuera-Cary).  FP64 without losses runs two workgroups per CU
// (two waves per SIMD, 256 registers; with losses that bound spills inside the loop)
// and FP32 three by its register count.  Both prefetch packets one quad round ahead;
// the FP64 loss variants, at one wave per SIMD, two rounds ahead.
template <typename T, bool LOSS>
constexpr bool two_wave_step() {
  return is_fp64<T>() && !LOSS;
}
template <typename T, bool LOSS>
constexpr int prefetch_depth() {
  return (is_fp64<T>() && LOSS) ? 2 : 1;
}

template <int M, typename T, bool DEP, bool LOSS, int PUSH>
__global__ void __launch_bounds__(kThreads, (two_wave_step<T, LOSS>() ? 2 : 1)) cells_step_kernel(StepView V, const T* __restrict__ E,
                                                              const T* __restrict__ B, const T* __restrict__ NN,
                                                              double* __restrict__ dM, double* __restrict__ dE,
                                                              RunConsts k) {
  constexpr int NF = LOSS ? 7 : 6;
  __shared__ T Fs[NF][kRegionCells];
  __shared__ double Acc[4][kRegionCells];
  __shared__ int cntB[kCellTileCells];
  __shared__ int cntD[kDirs];
  __shared__ int sDcap[kDirs];
  __shared__ int sDoff[kDirs + 1];
  __shared__ int sPre[kDirs + 1];   // prefix of this tile's inbox counts by direction
  __shared__ int sLo[kCellTileCells + 1];  // prefix of the packets left over past the round cap
  __shared__ int sR;                // round cap of the quad loop
  // per-wave exchange areas of the quad loop: per lane, the packet's weights and
  // exchange values (Pk) and the lane's partial field sums (Rs)
  __shared__ __attribute__((aligned(16))) T Pk[kThreads / 64][64 * kPkStride<T>];
  __shared__ __attribute__((aligned(16))) T Rs[kThreads / 64][64 * kRsStride<T>];

  constexpr bool deposit = DEP;
  const int64_t ntiles = V.ntiles;
  int tile = blockIdx.x;
  // consecutive workgroups go to different XCDs: give each XCD a contiguous range of
  // tiles so neighbouring tiles share that XCD's L2
  if ((ntiles & 7) == 0) tile = (int)(blockIdx.x & 7) * (int)(ntiles >> 3) + (int)(blockIdx.x >> 3);
  const int ttx = tile % V.ntx;
  const int tty = (tile / V.ntx) % V.nty;
  const int ttz = tile / (V.ntx * V.nty);
  const int ox = ttx * kCellTile - 1, oy = tty * kCellTile - 1, oz = ttz * kCellTile - 1;
  const int64_t nc = k.ncells;
  const int64_t trash = V.tr0 + (int)(blockIdx.x & 7) * kThreads + threadIdx.x;
  uint32_t err = 0;

  // this thread's quad, cell and first packets: every load of the prologue is issued
  // before the first wait, so a workgroup pays one memory latency before its loop
  const int q = threadIdx.x & 3;
  const int quad = threadIdx.x >> 2;
  const int lane = threadIdx.x & 63;
  const int lx = quad & 3, ly = (quad >> 2) & 3, lz = quad >> 4;
  const int home[3] = {ttx * kCellTile + lx, tty * kCellTile + ly, ttz * kCellTile + lz};
  const bool valid = home[0] < k.nx && home[1] < k.ny && home[2] < k.nz;
  const int64_t cell = valid ? home[0] + (int64_t)k.nx * (home[1] + (int64_t)k.ny * home[2]) : 0;
  const int n_raw = V.bcnt_in[cell];
  // the first wave also reads the counts of all 64 cells (lane = cell in tile)
  int64_t lcell = 0;
  bool lvalid = false;
  if (threadIdx.x < kCellTileCells) {
    const int gx = ttx * kCellTile + (threadIdx.x & 3), gy = tty * kCellTile + ((threadIdx.x >> 2) & 3),
              gz = ttz * kCellTile + (threadIdx.x >> 4);
    lvalid = gx < k.nx && gy < k.ny && gz < k.nz;
    lcell = lvalid ? gx + (int64_t)k.nx * (gy + (int64_t)k.ny * gz) : 0;
  }
  const int nl_raw = threadIdx.x < kCellTileCells ? V.bcnt_in[lcell] : 0;

  const SlotArrays& S = V.in;
  const T* su = (const T*)S.u;
  // packet state of the next rounds: one register set filled a round ahead (the other
  // waves of the SIMD cover the load latency, and the registers saved keep the FP64
  // loop free of spills: with two sets it spilled to scratch inside the loop, and its
  // reloads waited on every outstanding load), or, at one wave per SIMD, two sets used
  // alternately so that a load has two rounds to arrive.  The first rounds load
  // before the cell's count is known, whatever the slots hold (stale data the lane
  // ignores); in the loop a lane past its cell's count skips the load
  T pua[3], pub[3];
  using PX = typename std::conditional<is_fp64<T>(), double, float>::type;  // position or offset
  PX pxa[3], pxb[3];
  int32_t pida, pidb;
  T pwa = T(1), pwb = T(1);
  auto fetch = [&](int rd, PX (&px)[3], T (&pu)[3], int32_t& pid, T& pw) {
    int kk = 4 * rd + q;
    kk = kk < V.cap ? kk : V.cap - 1;
    const int64_t j = slot_index(tile, kk, quad, V.cap);
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      if constexpr (is_fp64<T>()) px[d] = S.x[d * S.stride + j];
      else px[d] = S.off[d * S.stride + j];
      pu[d] = su[d * S.stride + j];
    }
    pid = S.id[j];
    if constexpr (LOSS) pw = ((const T*)S.w)[j];
  };
  constexpr int kDepth = prefetch_depth<T, LOSS>();
  fetch(0, pxa, pua, pida, pwa);
  if constexpr (kDepth == 2) fetch(1, pxb, pub, pidb, pwb);
  // this tile's inbox counts by direction, one per lane of the first wave
  const int cin = threadIdx.x < kDirs ? V.icnt_in[(int64_t)tile * kDirs + threadIdx.x] : 0;

  for (int r = threadIdx.x; r < kRegionCells; r += kThreads) {
    const int rx = r % kRegionEdge, ry = (r / kRegionEdge) % kRegionEdge, rz = r / (kRegionEdge * kRegionEdge);
    const int64_t rc =
        wrapm(ox + rx, k.nx) + (int64_t)k.nx * (wrapm(oy + ry, k.ny) + (int64_t)k.ny * wrapm(oz + rz, k.nz));
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      Fs[d][r] = E[d * nc + rc];
      Fs[3 + d][r] = B[d * nc + rc];
    }
    if constexpr (LOSS) Fs[6][r] = NN[rc];
    if constexpr (deposit) {
      #pragma unroll
      for (int d = 0; d < 4; ++d) Acc[d][r] = 0.0;
    }
  }
  if (threadIdx.x < kCellTileCells) cntB[threadIdx.x] = 0;
  if (threadIdx.x < 64) {
    // part capacities and offsets by lane (uniform kernel-argument reads), then the
    // prefix of the clamped counts across the first wave
    int dcap = 0, doff = V.doff[kDirs];
    #pragma unroll
    for (int d = 0; d < kDirs; ++d) {
      dcap = threadIdx.x == d ? V.dcap[d] : dcap;
      doff = threadIdx.x == d ? V.doff[d] : doff;
    }
    if (threadIdx.x < kDirs) {
      cntD[threadIdx.x] = 0;
      sDcap[threadIdx.x] = dcap;
    }
    if (threadIdx.x <= kDirs) sDoff[threadIdx.x] = doff;
    const int c = cin < dcap ? cin : dcap;
    int incl = c;
    #pragma unroll
    for (int o = 1; o < 32; o <<= 1) {
      const int y = __shfl_up(incl, o);
      if (lane >= o) incl += y;
    }
    if (threadIdx.x <= kDirs) sPre[threadIdx.x] = incl - c;
    // round cap of the quad loop: the tile's mean rounds per cell, rounded up; a
    // cell's packets past it are left to the per-packet phase, which spreads them
    // over the whole workgroup instead of making every wave wait for the fullest cell
    int nl = lvalid ? (nl_raw < V.cap ? nl_raw : V.cap) : 0;
    int tot = nl;
    #pragma unroll
    for (int o = 1; o < 64; o <<= 1) tot += __shfl_xor(tot, o);
    const int R = (tot + 4 * kCellTileCells - 1) / (4 * kCellTileCells) + kRoundSlack;
    const int lo = nl > 4 * R ? nl - 4 * R : 0;
    int lincl = lo;
    #pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(lincl, o);
      if (lane >= o) lincl += y;
    }
    sLo[threadIdx.x] = lincl - lo;
    if (threadIdx.x == kCellTileCells - 1) {
      sLo[kCellTileCells] = lincl;
      sR = R > 0 ? R : 1;
    }
  }
  __syncthreads();

  const T h = (T)k.h, hb = (T)k.hb;
  const T pf = (T)k.pfac, ef = (T)k.efac;
  const T lrate = (T)k.lrate;

  // ------------------------------------------------------------ quads: one cell each
  {
    const int qbase = lane & ~3;  // first lane of this quad within the wave
    T* pkw = &Pk[threadIdx.x >> 6][0];
    T* rsw = &Rs[threadIdx.x >> 6][0];
    int n = valid ? n_raw : 0;
    n = n < V.cap ? n : V.cap;
    n = n < 4 * sR ? n : 4 * sR;  // packets past the round cap go to the per-packet phase

    // this lane's field components on the 27 nodes around the cell.  Without losses
    // the quad holds E_x, E_y, E_z, B_x in F0 (lane q: component q) and B_y, B_z, B_y,
    // B_z in F1, so the six components of its four packets take six passes: four over
    // F0 and two over F1, where lanes 0, 1 serve packets 0, 2 and lanes 2, 3 packets
    // 1, 3.  With losses lane q < 3 holds E_q, B_q and lane 3 the nucleon density.
    // With TSC the node values are turned into the interpolant's coefficients once
    // (tsc_coefficients) and each pass evaluates them at a packet's three offsets.
    T F0[27], F1[27], D[27];
    #pragma unroll
    for (int c = 0; c < 3; ++c)
      #pragma unroll
      for (int b = 0; b < 3; ++b)
        #pragma unroll
        for (int a = 0; a < 3; ++a) {
          const int node = a + 3 * (b + 3 * c);
          const int r = (lx + a) + kRegionEdge * ((ly + b) + kRegionEdge * (lz + c));
          if constexpr (LOSS) {
            F0[node] = q < 3 ? Fs[q][r] : Fs[6][r];
            F1[node] = q < 3 ? Fs[3 + q][r] : T(0);
          } else {
            F0[node] = Fs[q][r];
            F1[node] = Fs[4 + (q & 1)][r];
          }
          D[node] = T(0);
        }
    if constexpr (M == 3) {
      tsc_coefficients<T>(F0);
      tsc_coefficients<T>(F1);
    }

    const int rounds = (n + 3) >> 2;
    // the previous round's packet, stored at the start of the next round (just before
    // that round's prefetch) so that the loop never waits on its own fresh stores
    int64_t oj = trash, ojc = trash;
    double oxn[3] = {0.0, 0.0, 0.0};
    T ofn[3] = {T(0), T(0), T(0)}, oun[3] = {T(0), T(0), T(0)};
    T ow = T(1);
    int32_t oid = 0, ocell = 0;
    auto flush = [&]() {
      store_slot<T, LOSS>(V.out, oj, ojc, oxn, ofn, oun, ow, oid, ocell);
    };
    auto round = [&](const int rd, PX (&px)[3], T (&pu)[3], int32_t& pid, T& pw) {
      const bool act = 4 * rd + q < n;
      T f[3], u[3];
      double xa[3] = {0.0, 0.0, 0.0};
      const int32_t id = pid;
      const T wv = act ? pw : T(1);
      #pragma unroll
      for (int d = 0; d < 3; ++d) {
        if constexpr (is_fp64<T>()) {
          xa[d] = px[d];
          const double s = xa[d] * k.inv_dx;
          f[d] = act ? s - floor(s) : 0.5;
        } else {
          f[d] = act ? (T)px[d] : T(0.5);
        }
        u[d] = act ? pu[d] : T(0);
      }
      flush();
      if (4 * (rd + kDepth) + q < n) fetch(rd + kDepth, px, pu, pid, pw);

      // own weights -> LDS: x weights, then the nine y-z products
      {
        T wx[3], wy[3], wz[3];
        weights3<M, T>(f[0], wx);
        weights3<M, T>(f[1], wy);
        weights3<M, T>(f[2], wz);
        T* o = pkw + lane * kPkStride<T>;
        o[0] = wx[0];
        o[1] = wx[1];
        o[2] = wx[2];
        #pragma unroll
        for (int c = 0; c < 3; ++c)
          #pragma unroll
          for (int b = 0; b < 3; ++b) o[3 + b + 3 * c] = wy[b] * wz[c];
        if constexpr (M == 3) {
          // offsets from the cell centre for the polynomial gather (the exchange values
          // take these slots after the gather)
          o[12] = f[0] - T(0.5);
          o[13] = f[1] - T(0.5);
          o[14] = f[2] - T(0.5);
        }
      }
      wave_sync();

      // gather: each lane sums its components over the 27 nodes for the packets it
      // serves and leaves the sums in LDS for the owner lanes
      T eb[6];
      if constexpr (LOSS) {
        #pragma unroll
        for (int J = 0; J < 4; ++J) {
          const T* wj = pkw + (qbase + J) * kPkStride<T>;
          if constexpr (M == 3) {
            const T dv[3] = {wj[12], wj[13], wj[14]};
            rsw[lane * kRsStride<T> + 2 * J] = tsc_poly<T>(dv, F0);
            rsw[lane * kRsStride<T> + 2 * J + 1] = tsc_poly<T>(dv, F1);
          } else {
            T w[12];
            #pragma unroll
            for (int i = 0; i < 12; ++i) w[i] = wj[i];
            rsw[lane * kRsStride<T> + 2 * J] = stencil_sum<T>(w, F0);
            rsw[lane * kRsStride<T> + 2 * J + 1] = stencil_sum<T>(w, F1);
          }
        }
        wave_sync();
        #pragma unroll
        for (int c = 0; c < 3; ++c) {
          eb[c] = rsw[(qbase + c) * kRsStride<T> + 2 * q];
          eb[3 + c] = rsw[(qbase + c) * kRsStride<T> + 2 * q + 1];
        }
      } else {
        #pragma unroll
        for (int J = 0; J < 4; ++J) {
          const T* wj = pkw + (qbase + J) * kPkStride<T>;
          if constexpr (M == 3) {
            const T dv[3] = {wj[12], wj[13], wj[14]};
            rsw[lane * kRsStride<T> + J] = tsc_poly<T>(dv, F0);
          } else {
            T w[12];
            #pragma unroll
            for (int i = 0; i < 12; ++i) w[i] = wj[i];
            rsw[lane * kRsStride<T> + J] = stencil_sum<T>(w, F0);
          }
        }
        #pragma unroll
        for (int p = 0; p < 2; ++p) {
          const T* wj = pkw + (qbase + 2 * p + (q >> 1)) * kPkStride<T>;
          if constexpr (M == 3) {
            const T dv[3] = {wj[12], wj[13], wj[14]};
            rsw[lane * kRsStride<T> + 4 + p] = tsc_poly<T>(dv, F1);
          } else {
            T w[12];
            #pragma unroll
            for (int i = 0; i < 12; ++i) w[i] = wj[i];
            rsw[lane * kRsStride<T> + 4 + p] = stencil_sum<T>(w, F1);
          }
        }
        wave_sync();
        #pragma unroll
        for (int c = 0; c < 4; ++c) eb[c] = rsw[(qbase + c) * kRsStride<T> + q];
        const int hy = qbase + 2 * (q & 1);  // lane holding B_y for this lane's packet
        eb[4] = rsw[hy * kRsStride<T> + 4 + (q >> 1)];
        eb[5] = rsw[(hy + 1) * kRsStride<T> + 4 + (q >> 1)];
      }

      // kick (Eq. (11))
      const Kick<T> kq = kick<PUSH, T>(u[0], u[1], u[2], eb[0], eb[1], eb[2], eb[3], eb[4], eb[5], h, hb);
      const T un[3] = {u[0] + kq.dux, u[1] + kq.duy, u[2] + kq.duz};
      // losses: weight update; the exchange becomes the change of the weighted totals,
      // wn du - w lost u (momentum) and wn dgamma - w lost gamma (energy)
      T wn = wv, lost = T(0);
      if constexpr (LOSS) {
        const T nnp = rsw[(qbase + 3) * kRsStride<T> + 2 * q];
        loss_step<T>(un[0], un[1], un[2], nnp, lrate, wv, &wn, &lost);
      }

      // exchange (Eq. (12)) into the quad's registers, lane q taking component q
      if constexpr (deposit) {
        T* o = pkw + lane * kPkStride<T>;
        if constexpr (LOSS) {
          const T wl = wv * lost;
          o[12] = act ? pf * (wn * kq.dux - wl * u[0]) : T(0);
          o[13] = act ? pf * (wn * kq.duy - wl * u[1]) : T(0);
          o[14] = act ? pf * (wn * kq.duz - wl * u[2]) : T(0);
          o[15] = act ? ef * (wn * kq.dg - wl * kq.g0) : T(0);
        } else {
          o[12] = act ? pf * kq.dux : T(0);
          o[13] = act ? pf * kq.duy : T(0);
          o[14] = act ? pf * kq.duz : T(0);
          o[15] = act ? ef * kq.dg : T(0);
        }
        wave_sync();
        #pragma unroll
        for (int J = 0; J < 4; ++J) {
          const T* wj = pkw + (qbase + J) * kPkStride<T>;
          T w[12];
          #pragma unroll
          for (int i = 0; i < 12; ++i) w[i] = wj[i];
          const T mine = wj[12 + q];
          // the x weights scaled by this lane's exchange value: three products instead of
          // one per y-z pair
          const T wxq[3] = {w[0] * mine, w[1] * mine, w[2] * mine};
          #pragma unroll
          for (int c = 0; c < 3; ++c)
            #pragma unroll
            for (int b = 0; b < 3; ++b)
              #pragma unroll
              for (int a = 0; a < 3; ++a) D[a + 3 * (b + 3 * c)] += wxq[a] * w[3 + b + 3 * c];
        }
        // the accumulation happens here: left to itself the compiler sinks these FMAs
        // past the drift and the slot placement, keeping the 52 values read above live
        // across them (FP64 357 registers and one wave per SIMD, FP32 209 and two)
        #pragma unroll
        for (int i = 0; i < 27; ++i) asm volatile("" : "+v"(D[i]));
      }
      wave_sync();

      // drift, then take a slot in the next buffer; every lane stores (idle lanes into
      // the trash slots) so that each round issues the same memory operations
      int hn[3];
      const uint32_t e1 = drift3<T>(k, home, f, xa, un, hn, oxn, ofn);
      err |= act ? e1 : 0u;
      bool to_bucket = false;
      oj = act ? place(V, ttx, tty, ttz, cntB, cntD, sDcap, sDoff, hn, &to_bucket) : trash;
      if (oj < 0) oj = place_overflow(V, trash, err);
      ojc = to_bucket ? trash : oj;
      #pragma unroll
      for (int d = 0; d < 3; ++d) oun[d] = un[d];
      ow = wn;
      oid = id;
      ocell = hn[0] + k.nx * (hn[1] + k.ny * hn[2]);
    };
    for (int rd = 0; __ballot(rd < rounds) != 0; rd += 2) {
      round(rd, pxa, pua, pida, pwa);
      if (__ballot(rd + 1 < rounds) == 0) break;
      if constexpr (kDepth == 1) round(rd + 1, pxa, pua, pida, pwa);
      else round(rd + 1, pxb, pub, pidb, pwb);
    }
    flush();
    if (deposit && n > 0) {
      #pragma unroll
      for (int c = 0; c < 3; ++c)
        #pragma unroll
        for (int b = 0; b < 3; ++b)
          #pragma unroll
          for (int a = 0; a < 3; ++a) {
            const int r = (lx + a) + kRegionEdge * ((ly + b) + kRegionEdge * (lz + c));
            atomicAdd(&Acc[q][r], (double)D[a + 3 * (b + 3 * c)]);
          }
    }
  }

  // ------------------------------------------------------------ per packet: leftovers, then inbox
  {
    // one packet per thread: gather from the staged fields, deposit with LDS atomics
    auto process = [&](const int home[3], const T f[3], const double xa[3], const T u[3], T wv, int32_t id) {
      // region coordinates of node home-1 (these packets all live in this tile)
      const int bx = home[0] - ttx * kCellTile, by = home[1] - tty * kCellTile, bz = home[2] - ttz * kCellTile;
      T w[9];
      weights3<M, T>(f[0], w);
      weights3<M, T>(f[1], w + 3);
      weights3<M, T>(f[2], w + 6);
      T eb[NF];
      gather27<NF, T>(w, [&](int node, int d) {
        const int a = node % 3, b = (node / 3) % 3, c = node / 9;
        return Fs[d][(bx + a) + kRegionEdge * ((by + b) + kRegionEdge * (bz + c))];
      }, eb);
      const Kick<T> kq = kick<PUSH, T>(u[0], u[1], u[2], eb[0], eb[1], eb[2], eb[3], eb[4], eb[5], h, hb);
      const T un[3] = {u[0] + kq.dux, u[1] + kq.duy, u[2] + kq.duz};
      T wn = wv, lost = T(0);
      if constexpr (LOSS) loss_step<T>(un[0], un[1], un[2], eb[NF - 1], lrate, wv, &wn, &lost);
      if constexpr (deposit) {
        const T wl = wv * lost;
        const T qv[4] = {LOSS ? pf * (wn * kq.dux - wl * u[0]) : pf * kq.dux,
                         LOSS ? pf * (wn * kq.duy - wl * u[1]) : pf * kq.duy,
                         LOSS ? pf * (wn * kq.duz - wl * u[2]) : pf * kq.duz,
                         LOSS ? ef * (wn * kq.dg - wl * kq.g0) : ef * kq.dg};
        #pragma unroll
        for (int c = 0; c < 3; ++c)
          #pragma unroll
          for (int b = 0; b < 3; ++b) {
            const T wyz = w[3 + b] * w[6 + c];
            #pragma unroll
            for (int a = 0; a < 3; ++a) {
              const int r = (bx + a) + kRegionEdge * ((by + b) + kRegionEdge * (bz + c));
              const T W = w[a] * wyz;
              if (W != T(0)) {
                #pragma unroll
                for (int d = 0; d < 4; ++d) atomicAdd(&Acc[d][r], (double)(W * qv[d]));
              }
            }
          }
      }
      int hn[3];
      double xn[3];
      T fn[3];
      err |= drift3<T>(k, home, f, xa, un, hn, xn, fn);
      bool to_bucket = false;
      int64_t j2 = place(V, ttx, tty, ttz, cntB, cntD, sDcap, sDoff, hn, &to_bucket);
      if (j2 < 0) j2 = place_overflow(V, trash, err);
      store_slot<T, LOSS>(V.out, j2, to_bucket ? trash : j2, xn, fn, un, wn, id, hn[0] + k.nx * (hn[1] + k.ny * hn[2]));
    };
    const int nlo = sLo[kCellTileCells];
    const int nin = sPre[kDirs];
    const int R = sR;
    for (int i = threadIdx.x; i < nlo + nin; i += kThreads) {
      int home[3];
      T f[3], u[3];
      double xa[3] = {0.0, 0.0, 0.0};
      int32_t id;
      T wv = T(1);
      if (i < nlo) {
        // leftover packet: cell lc with sLo[lc] <= i < sLo[lc + 1], slot 4R + (i - sLo[lc])
        int lo = 0, hi = kCellTileCells - 1;
        while (lo < hi) {
          const int mid = (lo + hi + 1) >> 1;
          if (sLo[mid] <= i) lo = mid;
          else hi = mid - 1;
        }
        const int lc = lo;
        home[0] = ttx * kCellTile + (lc & 3);
        home[1] = tty * kCellTile + ((lc >> 2) & 3);
        home[2] = ttz * kCellTile + (lc >> 4);
        const int64_t j = slot_index(tile, 4 * R + (i - sLo[lc]), lc, V.cap);
        #pragma unroll
        for (int d = 0; d < 3; ++d) {
          if constexpr (is_fp64<T>()) {
            xa[d] = S.x[d * S.stride + j];
            const double sc = xa[d] * k.inv_dx;
            f[d] = sc - floor(sc);
          } else {
            f[d] = S.off[d * S.stride + j];
          }
          u[d] = su[d * S.stride + j];
        }
        id = S.id[j];
        if constexpr (LOSS) wv = ((const T*)S.w)[j];
      } else {
        const int ii = i - nlo;
        int dir = 0;
        #pragma unroll
        for (int d = 1; d < kDirs; ++d) dir += (ii >= sPre[d]) ? 1 : 0;
        const int64_t j = (int64_t)tile * V.per_tile + sDoff[dir] + (ii - sPre[dir]);
        load_free<T, LOSS>(V.in, V.ib0 + j, k, home, f, xa, u, wv, id);
      }
      process(home, f, xa, u, wv, id);
    }
  }

  // ------------------------------------------------------------ overflow list, shared by all workgroups
  {
    int nov = V.icnt_in[ntiles * kDirs];
    nov = (int64_t)nov < V.ocap ? nov : (int)V.ocap;
    const int n3[3] = {k.nx, k.ny, k.nz};
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < nov; i += (int64_t)gridDim.x * kThreads) {
      int home[3];
      T f[3], u[3];
      double xa[3];
      int32_t id;
      T wv;
      load_free<T, LOSS>(V.in, V.ov0 + i, k, home, f, xa, u, wv, id);
      T w[9];
      weights3<M, T>(f[0], w);
      weights3<M, T>(f[1], w + 3);
      weights3<M, T>(f[2], w + 6);
      int64_t nodes[27];
      #pragma unroll
      for (int c = 0; c < 3; ++c)
        #pragma unroll
        for (int b = 0; b < 3; ++b)
          #pragma unroll
          for (int a = 0; a < 3; ++a)
            nodes[a + 3 * (b + 3 * c)] = wrapm(home[0] - 1 + a, n3[0]) +
                (int64_t)k.nx * (wrapm(home[1] - 1 + b, n3[1]) + (int64_t)k.ny * wrapm(home[2] - 1 + c, n3[2]));
      T eb[NF];
      gather27<NF, T>(w, [&](int node, int d) {
        return d < 3 ? E[d * nc + nodes[node]] : (d < 6 ? B[(d - 3) * nc + nodes[node]] : NN[nodes[node]]);
      }, eb);
      const Kick<T> kq = kick<PUSH, T>(u[0], u[1], u[2], eb[0], eb[1], eb[2], eb[3], eb[4], eb[5], h, hb);
      const T un[3] = {u[0] + kq.dux, u[1] + kq.duy, u[2] + kq.duz};
      T wn = wv, lost = T(0);
      if constexpr (LOSS) loss_step<T>(un[0], un[1], un[2], eb[NF - 1], lrate, wv, &wn, &lost);
      if constexpr (deposit) {
        const T wl = wv * lost;
        const T qv[4] = {LOSS ? pf * (wn * kq.dux - wl * u[0]) : pf * kq.dux,
                         LOSS ? pf * (wn * kq.duy - wl * u[1]) : pf * kq.duy,
                         LOSS ? pf * (wn * kq.duz - wl * u[2]) : pf * kq.duz,
                         LOSS ? ef * (wn * kq.dg - wl * kq.g0) : ef * kq.dg};
        #pragma unroll
        for (int c = 0; c < 3; ++c)
          #pragma unroll
          for (int b = 0; b < 3; ++b)
            #pragma unroll
            for (int a = 0; a < 3; ++a) {
              const T W = w[a] * w[3 + b] * w[6 + c];
              if (W != T(0)) {
                const int64_t g = nodes[a + 3 * (b + 3 * c)];
                #pragma unroll
                for (int d = 0; d < 3; ++d) atomicAdd(&dM[d * nc + g], (double)(W * qv[d]));
                if (dE) atomicAdd(&dE[g], (double)(W * qv[3]));
              }
            }
      }
      int hn[3];
      double xn[3];
      T fn[3];
      err |= drift3<T>(k, home, f, xa, un, hn, xn, fn);
      const int64_t j2 = place_overflow(V, trash, err);
      store_slot<T, LOSS>(V.out, j2, j2, xn, fn, un, wn, id, hn[0] + k.nx * (hn[1] + k.ny * hn[2]));
    }
  }
  if (err) set_status(k.status, err);
  __syncthreads();

  // ------------------------------------------------------------ outputs
  if constexpr (deposit) {
    double* out = V.halo + (int64_t)tile * 4 * kRegionCells;
    const double* acc = &Acc[0][0];
    for (int r = threadIdx.x; r < 4 * kRegionCells; r += kThreads) out[r] = acc[r];
  }
  if (threadIdx.x < kCellTileCells) {
    const int lx = threadIdx.x & 3, ly = (threadIdx.x >> 2) & 3, lz = threadIdx.x >> 4;
    const int gx = ttx * kCellTile + lx, gy = tty * kCellTile + ly, gz = ttz * kCellTile + lz;
    if (gx < k.nx && gy < k.ny && gz < k.nz) {
      const int v = cntB[threadIdx.x];
      V.bcnt_out[gx + (int64_t)k.nx * (gy + (int64_t)k.ny * gz)] = v < V.cap ? v : V.cap;
    }
  } else if (threadIdx.x >= 64 && threadIdx.x < 64 + kDirs) {
    // count of part `dir` of the inbox of the tile at offset dir; this workgroup is
    // that part's only writer
    const int dir = threadIdx.x - 64;
    const int sx = dir % 3 - 1, sy = (dir / 3) % 3 - 1, sz = dir / 9 - 1;
    const int64_t t = wrapm(ttx + sx, V.ntx) +
                      (int64_t)V.ntx * (wrapm(tty + sy, V.nty) + (int64_t)V.nty * wrapm(ttz + sz, V.ntz));
    const int v = cntD[dir];
    V.icnt_out[t * kDirs + dir] = v < sDcap[dir] ? v : sDcap[dir];
  }
}

// After a step: add the per-tile exchange accumulators into the grid (a cell takes
// every region slot, of its own tile and of neighbouring tiles' halos, that maps onto
// it) and clear the overflow counter of the buffer the step consumed.  In a coupled
// step dM, dE are the gas momentum and energy, and the cell's E is refreshed from the
// updated momentum.
__global__ void cells_post_kernel(StepView V, double* dM, double* dE, GasLink gas, RunConsts k) {
  const int64_t nc = k.ncells;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (blockIdx.x == 0 && threadIdx.x == 0) V.icnt_in[V.ntiles * kDirs] = 0;
  if (!dM) return;
  const int n3[3] = {k.nx, k.ny, k.nz};
  const int nt[3] = {V.ntx, V.nty, V.ntz};
  // whole tiles and at least three of them along every axis: a cell's slots are its own
  // tile's and, on a tile face, the neighbour's across it (no wrap folds two together)
  bool whole = true;
  #pragma unroll
  for (int d = 0; d < 3; ++d) whole &= n3[d] % kCellTile == 0 && nt[d] >= 3;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nc; c += stride) {
    const int g[3] = {(int)(c % k.nx), (int)((c / k.nx) % k.ny), (int)(c / ((int64_t)k.nx * k.ny))};
    // per axis: (tile, region index) pairs whose region slot is this cell, in the order
    // of the tiles before, at and after the cell's own
    int tl[3][8], rl[3][8], cnt[3] = {0, 0, 0};
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int t0 = g[d] / kCellTile;
      if (whole) {
        const int l = g[d] - t0 * kCellTile;
        if (l == 0) {
          tl[d][0] = t0 == 0 ? nt[d] - 1 : t0 - 1;
          rl[d][0] = kRegionEdge - 1;
          tl[d][1] = t0;
          rl[d][1] = 1;
          cnt[d] = 2;
        } else if (l == kCellTile - 1) {
          tl[d][0] = t0;
          rl[d][0] = l + 1;
          tl[d][1] = t0 == nt[d] - 1 ? 0 : t0 + 1;
          rl[d][1] = 0;
          cnt[d] = 2;
        } else {
          tl[d][0] = t0;
          rl[d][0] = l + 1;
          cnt[d] = 1;
        }
        continue;
      }
      for (int dt = -1; dt <= 1; ++dt) {
        const int t = wrapm(t0 + dt, nt[d]);
        bool dup = false;
        for (int e = 0; e < cnt[d]; ++e) dup |= tl[d][e] == t;
        if (dup) continue;
        for (int r = 0; r < kRegionEdge; ++r)
          if (wrapm(t * kCellTile - 1 + r, n3[d]) == g[d] && cnt[d] < 8) {
            tl[d][cnt[d]] = t;
            rl[d][cnt[d]] = r;
            ++cnt[d];
          }
      }
    }
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int a = 0; a < cnt[0]; ++a)
      for (int b = 0; b < cnt[1]; ++b)
        for (int e = 0; e < cnt[2]; ++e) {
          const int64_t t = tl[0][a] + (int64_t)V.ntx * (tl[1][b] + (int64_t)V.nty * tl[2][e]);
          const int r = rl[0][a] + kRegionEdge * (rl[1][b] + kRegionEdge * rl[2][e]);
          const double* src = V.halo + t * 4 * kRegionCells + r;
          #pragma unroll
          for (int d = 0; d < 4; ++d) s[d] += src[d * kRegionCells];
        }
    dM[c] += s[0];
    dM[nc + c] += s[1];
    dM[2 * nc + c] += s[2];
    if (dE) dE[c] += s[3];
    if (gas.rho) gas_refresh(gas, c, nc);
  }
}

// Slot of this lane in a per-key counter, one atomic per run of equal keys among
// consecutive lanes (keys < 0 take no slot).
__device__ __forceinline__ int run_slot(int32_t* counters, int key) {
  const int lane = __lane_id();
  const int prev = __shfl_up(key, 1);
  const bool head = (lane == 0) || (prev != key);
  const unsigned long long heads = __ballot(head);
  const unsigned long long upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
  const int start = 63 - __clzll(heads & upto);
  const unsigned long long after = heads & ~upto;
  const int end = after ? (__ffsll((long long)after) - 1) : 64;
  int base = 0;
  if (lane == start && key >= 0) base = atomicAdd(&counters[key], end - start);
  base = __shfl(base, start);
  return key >= 0 ? base + (lane - start) : -1;
}

// Caller packets -> buffer 0: bucket slot from a per-cell counter, else the self part
// of the tile's inbox, else the overflow list.
template <typename T>
__global__ void __launch_bounds__(kThreads) cells_build_kernel(Packets<T> P, CellLists L, RunConsts k) {
  const int n3[3] = {k.nx, k.ny, k.nz};
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < P.np; base += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = base + threadIdx.x;
    int key = -1;
    int h[3] = {0, 0, 0};
    T f[3] = {T(0), T(0), T(0)}, u[3] = {T(0), T(0), T(0)};
    double x[3] = {0.0, 0.0, 0.0};
    if (i < P.np) {
      if constexpr (is_fp64<T>()) {
        #pragma unroll
        for (int d = 0; d < 3; ++d) {
          x[d] = P.x[d * P.np + i];
          h[d] = wrapm((int)floor(x[d] * k.inv_dx), n3[d]);
        }
      } else {
        int c = P.cell[i];
        c = c < 0 ? 0 : (c >= k.ncells ? k.ncells - 1 : c);
        cell_coords(c, k, h);
        #pragma unroll
        for (int d = 0; d < 3; ++d) f[d] = P.off[d * P.np + i];
      }
      #pragma unroll
      for (int d = 0; d < 3; ++d) u[d] = P.u[d * P.np + i];
      key = h[0] + k.nx * (h[1] + k.ny * h[2]);
    }
    const int slot = run_slot(L.bcnt[0], key);
    if (i >= P.np) continue;
    const int32_t id = P.id[i];
    const int64_t trash = L.tr0 + (blockIdx.x & 7) * kThreads + threadIdx.x;
    int64_t j, jc;
    if (slot < L.cap) {
      j = bucket_index(h, slot, L.ntx, L.nty, L.cap);
      jc = trash;
    } else {
      const int64_t t = h[0] / kCellTile + (int64_t)L.ntx * (h[1] / kCellTile + (int64_t)L.nty * (h[2] / kCellTile));
      const int is = atomicAdd(&L.icnt[0][t * kDirs + kSelfDir], 1);
      if (is < L.dcap[kSelfDir]) {
        j = L.ib0 + t * L.per_tile + L.doff[kSelfDir] + is;
      } else {
        const int os = atomicAdd(&L.icnt[0][L.ntiles * kDirs], 1);
        if ((int64_t)os >= L.ocap) {
          set_status(k.status, ERR_TILE);
          continue;
        }
        j = L.ov0 + os;
      }
      jc = j;
    }
    store_slot<T, false>(L.buf[0], j, jc, x, f, u, T(1), id, key);
    if (P.w && L.buf[0].w) ((T*)L.buf[0].w)[j] = P.w[i];
  }
}

// Clamped occupancy of every store, in compaction order: cells, tile directions, overflow.
__global__ void cells_counts_kernel(CellLists L, int64_t nc, int32_t* __restrict__ out) {
  const int cur = L.cur;
  const int64_t ni = L.ntiles * kDirs;
  const int64_t n = nc + ni + 1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int v, cap;
    if (i < nc) {
      v = L.bcnt[cur][i];
      cap = L.cap;
    } else if (i < nc + ni) {
      v = L.icnt[cur][i - nc];
      const int dir = (int)((i - nc) % kDirs);
      cap = 0;
      #pragma unroll
      for (int d = 0; d < kDirs; ++d) cap = (dir == d) ? L.dcap[d] : cap;
    } else {
      v = L.icnt[cur][ni];
      cap = (int)L.ocap;
    }
    out[i] = v < cap ? v : cap;
  }
}

template <typename T>
__device__ __forceinline__ void copy_out(const Packets<T>& P, const SlotArrays& S, int64_t j, int64_t o,
                                         int32_t cell) {
  const T* su = (const T*)S.u;
  #pragma unroll
  for (int d = 0; d < 3; ++d) {
    if constexpr (is_fp64<T>()) P.x[d * P.np + o] = S.x[d * S.stride + j];
    else P.off[d * P.np + o] = S.off[d * S.stride + j];
    P.u[d * P.np + o] = su[d * S.stride + j];
  }
  if constexpr (!is_fp64<T>()) P.cell[o] = cell;
  P.id[o] = S.id[j];
  if (P.w && S.w) P.w[o] = ((const T*)S.w)[j];
}

// The buckets of buffer cur -> caller arrays, one wave per cell: the lanes take the
// cell's slots and write its contiguous output range.  A workgroup's 16 waves take the
// 16 cells of one z-plane of a tile, whose slots share the lines of each slot row, so a
// line is read by the waves together.
constexpr int kCompactThreads = 1024;
template <typename T>
__global__ void __launch_bounds__(kCompactThreads) cells_compact_buckets_kernel(Packets<T> P, CellLists L,
                                                                                const int32_t* __restrict__ offs,
                                                                                RunConsts k) {
  const SlotArrays& S = L.buf[L.cur];
  const int64_t t = blockIdx.x / kCellTile;
  const int lz = (int)(blockIdx.x - t * kCellTile);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;  // w = lx + 4 ly
  const int lc = w + kCellTile * kCellTile * lz;
  const int gx = (int)(t % L.ntx) * kCellTile + (w & 3), gy = (int)((t / L.ntx) % L.nty) * kCellTile + (w >> 2),
            gz = (int)(t / ((int64_t)L.ntx * L.nty)) * kCellTile + lz;
  if (gx >= k.nx || gy >= k.ny || gz >= k.nz) return;
  const int64_t c = gx + (int64_t)k.nx * (gy + (int64_t)k.ny * gz);
  const int n = offs[c + 1] - offs[c];  // clamped to the bucket capacity by the counts
  for (int sl = lane; sl < n; sl += 64) copy_out<T>(P, S, slot_index(t, sl, lc, L.cap), offs[c] + sl, (int32_t)c);
}

// The inbox parts and the overflow list of buffer cur -> caller arrays at their
// prefix-sum offsets (each part's slots write one contiguous run).
template <typename T>
__global__ void cells_compact_kernel(Packets<T> P, CellLists L, const int32_t* __restrict__ offs, RunConsts k) {
  const SlotArrays& S = L.buf[L.cur];
  const int64_t nc = k.ncells;
  const int64_t nslot = L.ib0, islots = L.ov0 - L.ib0;
  const int64_t total = L.ov0 + L.ocap;
  const int64_t obase = nc + L.ntiles * kDirs;
  for (int64_t s = nslot + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < total;
       s += (int64_t)gridDim.x * blockDim.x) {
    if (s < nslot + islots) {
      const int64_t si = s - nslot;
      const int64_t t = si / L.per_tile;
      const int r = (int)(si - t * L.per_tile);
      int dir = 0, start = 0;
      #pragma unroll
      for (int d = 1; d < kDirs; ++d)
        if (r >= L.doff[d]) {
          dir = d;
          start = L.doff[d];
        }
      const int sl = r - start;
      const int64_t e = nc + t * kDirs + dir;
      if (sl >= offs[e + 1] - offs[e]) continue;
      const int32_t cell = is_fp64<T>() ? 0 : S.cell[s];
      copy_out<T>(P, S, s, offs[e] + sl, cell);
    } else {
      const int64_t so = s - nslot - islots;
      if (so >= offs[obase + 1] - offs[obase]) continue;
      const int32_t cell = is_fp64<T>() ? 0 : S.cell[s];
      copy_out<T>(P, S, s, offs[obase] + so, cell);
    }
  }
}

// offs[n] = offs[n-1] + counts[n-1] (total of an exclusive scan of n counts)
__global__ void scan_total_kernel(int32_t* offs, const int32_t* counts, int64_t n) {
  offs[n] = offs[n - 1] + counts[n - 1];
}

__global__ void zero_i32(int32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

inline int grid_for(int64_t n) {
  int64_t g = (n + kThreads - 1) / kThreads;
  return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

// Bump allocator over a (possibly notional) base address; every piece 256-aligned.
struct Carver {
  uintptr_t p;
  char* take(size_t n) {
    char* at = (char*)p;
    p += (n + 255) / 256 * 256;
    return at;
  }
};

SlotArrays carve_slots(Carver& cv, int64_t nslots, bool f32, bool with_cell, bool weights) {
  SlotArrays S;
  S.stride = nslots;
  const size_t n = (size_t)nslots;
  S.x = f32 ? nullptr : (double*)cv.take(3 * n * sizeof(double));
  S.off = f32 ? (float*)cv.take(3 * n * sizeof(float)) : nullptr;
  S.cell = (f32 && with_cell) ? (int32_t*)cv.take(n * sizeof(int32_t)) : nullptr;
  S.u = (void*)cv.take(3 * n * (f32 ? sizeof(float) : sizeof(double)));
  S.id = (int32_t*)cv.take(n * sizeof(int32_t));
  S.w = weights ? (void*)cv.take(n * (f32 ? sizeof(float) : sizeof(double))) : nullptr;
  return S;
}

CellLists carve(int nx, int ny, int nz, int64_t np, int precision, bool weights, uintptr_t base, size_t* bytes) {
  CellLists L;
  const int64_t ncells = (int64_t)nx * ny * nz;
  L.ntx = (nx + kCellTile - 1) / kCellTile;
  L.nty = (ny + kCellTile - 1) / kCellTile;
  L.ntz = (nz + kCellTile - 1) / kCellTile;
  L.ntiles = (int64_t)L.ntx * L.nty * L.ntz;
  // a cell holds Poisson-like counts around the mean: twice the mean plus a margin
  // keeps bucket overflow rare.  Inbox parts by the number of tile faces crossed:
  // self (full buckets) and faces take four buckets' worth, edges one, corners a
  // quarter.
  const int64_t mean = (np + ncells - 1) / ncells;
  L.cap = (int)((2 * mean + 16 + kSlotGroup - 1) / kSlotGroup * kSlotGroup);
  int off = 0;
  for (int d = 0; d < kDirs; ++d) {
    const int axes = (d % 3 != 1) + ((d / 3) % 3 != 1) + (d / 9 != 1);
    const int c = axes <= 1 ? 4 * L.cap : axes == 2 ? L.cap : L.cap / 4 + 8;
    L.dcap[d] = c;
    L.doff[d] = off;
    off += c;
  }
  L.doff[kDirs] = off;
  L.per_tile = off;
  L.ocap = np > 0 ? np : 1;
  const bool f32 = precision == 1;
  Carver cv{(base + 255) / 256 * 256};
  const uintptr_t start = cv.p;
  L.ib0 = L.ntiles * L.cap * kCellTileCells;
  L.ov0 = L.ib0 + L.ntiles * L.per_tile;
  L.tr0 = L.ov0 + L.ocap;
  const int64_t slots = L.tr0 + kTrashSlots;
  for (int b = 0; b < 2; ++b) {
    L.buf[b] = carve_slots(cv, slots, f32, true, weights);
    L.bcnt[b] = (int32_t*)cv.take((size_t)ncells * sizeof(int32_t));
    L.icnt[b] = (int32_t*)cv.take((size_t)(L.ntiles * kDirs + 1) * sizeof(int32_t));
  }
  L.halo = (double*)cv.take((size_t)L.ntiles * 4 * kRegionCells * sizeof(double));
  const int64_t nscan = ncells + L.ntiles * kDirs + 1;
  // counts (nscan), offsets (nscan + 1), scan temporaries
  L.scan = (int32_t*)cv.take((size_t)(2 * nscan + 1 + (int64_t)exclusive_scan_tmp_ints(nscan)) * sizeof(int32_t));
  L.cur = 0;
  if (bytes) *bytes = (size_t)(cv.p - start) + 256;
  return L;
}

}  // namespace

size_t cell_list_bytes(int nx, int ny, int nz, int64_t np, int precision, bool weights) {
  size_t bytes = 0;
  (void)carve(nx, ny, nz, np, precision, weights, 0, &bytes);
  return bytes;
}

CellLists cell_list_carve(int nx, int ny, int nz, int64_t np, int precision, bool weights, char* base) {
  return carve(nx, ny, nz, np, precision, weights, (uintptr_t)base, nullptr);
}

int64_t cell_list_scan_entries(int nx, int ny, int nz) {
  const int64_t nt = (int64_t)((nx + kCellTile - 1) / kCellTile) * ((ny + kCellTile - 1) / kCellTile) *
                     ((nz + kCellTile - 1) / kCellTile);
  return (int64_t)nx * ny * nz + nt * kDirs + 1;
}

template <typename T>
hipError_t launch_cells_build(const Packets<T>& P, CellLists& L, const RunConsts& k, hipStream_t s) {
  L.cur = 0;
  const int64_t ni = L.ntiles * kDirs + 1;
  hipLaunchKernelGGL(zero_i32, dim3(grid_for(k.ncells)), dim3(kThreads), 0, s, L.bcnt[0], (int64_t)k.ncells);
  hipLaunchKernelGGL(zero_i32, dim3(grid_for(ni)), dim3(kThreads), 0, s, L.icnt[0], ni);
  hipLaunchKernelGGL(zero_i32, dim3(grid_for(ni)), dim3(kThreads), 0, s, L.icnt[1], ni);
  if (P.np > 0) hipLaunchKernelGGL(cells_build_kernel<T>, dim3(grid_for(P.np)), dim3(kThreads), 0, s, P, L, k);
  return hipGetLastError();
}

// One launch of the step kernel for the run's pusher.
template <int M, typename T, bool D, bool L>
void launch_cells_variant(const StepView& V, const T* E, const T* B, const T* NN, double* dM, double* dE,
                          const RunConsts& k, hipStream_t s) {
  const dim3 grid((unsigned)V.ntiles), block(kThreads);
  if (k.pusher == kPushVay)
    hipLaunchKernelGGL((cells_step_kernel<M, T, D, L, kPushVay>), grid, block, 0, s, V, E, B, NN, dM, dE, k);
  else if (k.pusher == kPushHC)
    hipLaunchKernelGGL((cells_step_kernel<M, T, D, L, kPushHC>), grid, block, 0, s, V, E, B, NN, dM, dE, k);
  else
    hipLaunchKernelGGL((cells_step_kernel<M, T, D, L, kPushBoris>), grid, block, 0, s, V, E, B, NN, dM, dE, k);
}

template <typename T>
hipError_t launch_cells_step(int shape, CellLists& L, const T* E, const T* B, const T* NN, double* dM, double* dE,
                             const GasLink& gas, const RunConsts& k, hipStream_t s, hipEvent_t before,
                             hipEvent_t after) {
  const StepView V = step_view(L);
  if (NN && !(L.buf[0].w && L.buf[1].w)) return hipErrorInvalidValue;
  if (before) (void)hipEventRecord(before, s);
  const bool dep = dM != nullptr, loss = NN != nullptr;
  if (shape == kShapeCIC) {
    if (loss) {
      if (dep) launch_cells_variant<2, T, true, true>(V, E, B, NN, dM, dE, k, s);
      else launch_cells_variant<2, T, false, true>(V, E, B, NN, dM, dE, k, s);
    } else {
      if (dep) launch_cells_variant<2, T, true, false>(V, E, B, NN, dM, dE, k, s);
      else launch_cells_variant<2, T, false, false>(V, E, B, NN, dM, dE, k, s);
    }
  } else {
    if (loss) {
      if (dep) launch_cells_variant<3, T, true, true>(V, E, B, NN, dM, dE, k, s);
      else launch_cells_variant<3, T, false, true>(V, E, B, NN, dM, dE, k, s);
    } else {
      if (dep) launch_cells_variant<3, T, true, false>(V, E, B, NN, dM, dE, k, s);
      else launch_cells_variant<3, T, false, false>(V, E, B, NN, dM, dE, k, s);
    }
  }
  if (after) (void)hipEventRecord(after, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t work = dM ? (int64_t)k.ncells : 1;
  hipLaunchKernelGGL(cells_post_kernel, dim3(grid_for(work)), dim3(kThreads), 0, s, V, dM, dE, gas, k);
  L.cur = 1 - L.cur;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cells_compact(const Packets<T>& P, CellLists& L, const RunConsts& k, hipStream_t s) {
  const int64_t nc = k.ncells;
  const int64_t nscan = nc + L.ntiles * kDirs + 1;
  int32_t* counts = L.scan;
  int32_t* offs = counts + nscan;
  int32_t* tmp = offs + nscan + 1;
  hipLaunchKernelGGL(cells_counts_kernel, dim3(grid_for(nscan)), dim3(kThreads), 0, s, L, nc, counts);
  hipError_t e = launch_exclusive_scan(counts, offs, nscan, tmp, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scan_total_kernel, dim3(1), dim3(1), 0, s, offs, counts, nscan);
  const int64_t total = L.ov0 + L.ocap;
  if (L.ntiles > 0)
    hipLaunchKernelGGL(cells_compact_buckets_kernel<T>, dim3((unsigned)(L.ntiles * kCellTile)), dim3(kCompactThreads),
                       0, s, P, L, offs, k);
  hipLaunchKernelGGL(cells_compact_kernel<T>, dim3(grid_for(total - L.ib0)), dim3(kThreads), 0, s, P, L, offs, k);
  return hipGetLastError();
}

#define RSOL_CELLS_INSTANTIATE(T)                                                                                  \
  template hipError_t launch_cells_build<T>(const Packets<T>&, CellLists&, const RunConsts&, hipStream_t);         \
  template hipError_t launch_cells_step<T>(int, CellLists&, const T*, const T*, const T*, double*, double*,        \
                                           const GasLink&, const RunConsts&, hipStream_t, hipEvent_t, hipEvent_t); \
  template hipError_t launch_cells_compact<T>(const Packets<T>&, CellLists&, const RunConsts&, hipStream_t);

RSOL_CELLS_INSTANTIATE(double)
RSOL_CELLS_INSTANTIATE(float)

}  // namespace rsol
