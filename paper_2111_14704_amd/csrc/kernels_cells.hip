// Cell-list fused packet step.
//
// Packets live in per-cell buckets (two ping-pong buffers), per-tile inboxes and one
// overflow list for the grid.  One 256-thread workgroup owns a 4x4x4 tile; each of
// its 64 cells is owned by a quad (4 lanes).  A quad keeps the field stencil of its
// cell in registers (the 27 node values of its components, as the coefficients of
// the TSC interpolant) and the cell's exchange deposit on the same 27 nodes (lane q:
// component q of dM_x, dM_y, dM_z, dE).  The cell's packets are taken four at a time,
// one per lane; the weights, offsets, exchange values and partial field sums of the
// four packets pass between the quad's lanes through a per-wave LDS area, so the
// main loop neither reads the field grid nor issues atomics to global memory.
//
// A bucket holds only packets that stayed in their cell: after its drift a packet
// still in its cell is written to the next bucket of the same cell, at the quad's
// running count (a ballot over the quad's lanes, no atomics), so every cell writes
// one ordered stream.  Every other packet goes to an inbox part of its new tile:
// part dir of tile t holds packets that came from tile t - dir (the self part holds
// packets that moved within the tile, and bucket overflow), and that tile is the
// part's only writer (slots from an LDS counter, the final count stored with a plain
// store).  At the start of the next step the workgroup lists its inbox packets by
// cell in LDS, and each quad takes its cell's inbox packets after its bucket in the
// same loop.  Quads are given cells in order of their packet counts, so the cells of
// a wave have similar counts and few lanes idle.  Packets that find their part full
// go to the overflow list (gather from global memory, global atomics); inbox packets
// beyond the LDS list take a per-packet path (gather from LDS-staged fields, LDS
// atomics).  The workgroup's exchange accumulator (tile plus one-cell halo) goes to a
// per-tile buffer, summed over the steps of one call, which a second kernel adds into
// the grid.
//
// A slot store holds one packet record per slot (plus id and weight arrays), addressed
// from base pointers in scalar registers: records by 64-bit byte offsets, the 4- and
// 8-byte arrays by 32-bit ones (the host checks that those stay below 4 GiB).
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
constexpr int kQueue = 1024;  // inbox packets per tile listed by cell in LDS

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

// Layout of the quad loop's LDS exchange areas, chosen against gfx950's measured bank
// behaviour: reads of 4 bytes go through 32 banks, 32 lanes at a time; reads of 8 bytes
// through 64 banks, 32 lanes at a time; reads of 12 or 16 bytes through 64 banks, 16
// lanes at a time; writes and atomics through 32 banks, 32, 16 or 8 lanes at a time for
// 4, 8 or 16 bytes.  Pk holds per lane 16 values (12 weights, then the 3 offsets that
// the 4 exchange values replace) at lane pitch kPkLane within a quad and quad pitch
// kPkQuad (elements): with 24 / 100 (FP32) and 20 / 82 (FP64) the lanes' own 16-byte
// writes, the quads' broadcast reads and the per-lane reads of one exchange value
// each fall on distinct banks.  Rs holds per lane up to 8 partial sums at an odd
// pitch, so that its writes and the reads in which each lane of a quad takes one value
// from each of its quad's lanes meet no conflict either.
template <typename T>
constexpr int kPkLane = sizeof(T) == 8 ? 20 : 24;
template <typename T>
constexpr int kPkQuad = sizeof(T) == 8 ? 82 : 100;
constexpr int kRsStride = 9;
// Offset in a wave's Pk area of the values of wave lane L.
template <typename T>
__device__ __forceinline__ int pk_at(int L) {
  return (L >> 2) * kPkQuad<T> + (L & 3) * kPkLane<T>;
}
// Pitch (doubles) of one component of the tail's exchange accumulator: 8 dwords apart
// modulo the 32 banks, so that the four lanes of a quad, adding the four components of
// one node, never meet in a bank.
constexpr int kAccPitch = kRegionCells + 4;

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
// per-packet paths' gather.
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
// reads one group of each of its wave's 16 cells (whole cache lines), and the stayers
// a cell writes in a round go to one or two groups of its own stream.  All slot
// indices fit 32 bits (checked on the host).
__device__ __forceinline__ uint32_t slot32(uint32_t t, uint32_t s, uint32_t lc, uint32_t cap) {
  return ((t * (cap / kSlotGroup) + (s >> 2)) * kCellTileCells + lc) * kSlotGroup + (s & 3u);
}

// Bucket slot s of the cell with grid coordinates h (64-bit, for the filing kernel).
__device__ __forceinline__ int64_t bucket_index(const int h[3], int s, int ntx, int nty, int cap) {
  const int tx = h[0] / kCellTile, ty = h[1] / kCellTile, tz = h[2] / kCellTile;
  const int64_t t = tx + (int64_t)ntx * (ty + (int64_t)nty * tz);
  const int lc = (h[0] - tx * kCellTile) + kCellTile * ((h[1] - ty * kCellTile) + kCellTile * (h[2] - tz * kCellTile));
  return ((t * (cap / kSlotGroup) + s / kSlotGroup) * kCellTileCells + lc) * kSlotGroup + s % kSlotGroup;
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
  int64_t ib0, ov0;
  int dcap[kParts];
  int doff[kParts + 1];
  SlotArrays in, out;
  const int32_t* bcnt_in;
  int32_t* bcnt_out;
  int32_t* icnt_in;   // [ntiles*kParts] then the overflow count
  int32_t* icnt_out;
  double* halo;
  int accumulate;     // add the step's exchange to the per-tile buffer (else overwrite it)
};

StepView step_view(const CellLists& L, bool accumulate) {
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
  for (int d = 0; d < kParts; ++d) V.dcap[d] = L.dcap[d];
  for (int d = 0; d <= kParts; ++d) V.doff[d] = L.doff[d];
  V.in = L.buf[a];
  V.out = L.buf[b];
  V.bcnt_in = L.bcnt[a];
  V.bcnt_out = L.bcnt[b];
  V.icnt_in = L.icnt[a];
  V.icnt_out = L.icnt[b];
  V.halo = L.halo;
  V.accumulate = accumulate ? 1 : 0;
  return V;
}

// One slot store, addressed by a slot index j: part a, b (and c) of record j sits at
// base + kRec j (a, b, c being the record array plus 0, 16, 32 bytes), element j of
// the 4- or 8-byte arrays at base + 4 j or base + 8 j (below 4 GiB).
template <typename T>
struct Slots {
  char* a;   // FP64: {x, y}; FP32: {off_x, off_y, off_z, id}
  char* b;   // FP64: {z, u_x}; FP32: {u_x, u_y, u_z, home cell}
  char* c;   // FP64: {u_y, u_z}
  char* id;  // FP64: int32
  char* w;   // packet weights (precision type), NULL without
};

template <typename T>
__device__ __forceinline__ Slots<T> slots_of(const SlotArrays& S) {
  Slots<T> P;
  P.a = (char*)S.a;
  P.b = (char*)S.b;
  P.c = (char*)S.c;
  P.id = (char*)S.id;
  P.w = (char*)S.w;
  return P;
}

// Byte offset of element j of size s (32-bit product, zero-extended).
__device__ __forceinline__ size_t boff(uint32_t j, uint32_t s) { return (size_t)(j * s); }

template <typename X>
__device__ __forceinline__ X ld(const char* base, uint32_t j) {
  return *(const X*)(base + boff(j, sizeof(X)));
}
template <typename X>
__device__ __forceinline__ void st(char* base, uint32_t j, X v) {
  *(X*)(base + boff(j, sizeof(X))) = v;
}

// Bytes of a slot's packet record (FP32 {off, id}, {u, cell}; FP64 {x, y}, {z, u_x},
// {u_y, u_z}): one record per slot, so that a packet moved alone fills whole 32-byte
// sectors (FP32) or nearly (FP64).  Records are addressed with 64-bit byte offsets.
template <typename T>
constexpr uint32_t kRec = is_fp64<T>() ? 48u : 32u;
// Part `base` (a, b or c: the record plus 0, 16 or 32 bytes) of slot j's record.
template <typename X, typename T>
__device__ __forceinline__ X ldr(const char* base, uint32_t j) {
  return *(const X*)(base + (size_t)j * kRec<T>);
}
template <typename X, typename T>
__device__ __forceinline__ void str(char* base, uint32_t j, X v) {
  *(X*)(base + (size_t)j * kRec<T>) = v;
}

// The packet of slot j: position (FP64 absolute x) or in-cell offset (FP32), momentum,
// id, and (FP32) the home cell the slot records.
template <typename T>
__device__ __forceinline__ void load_packet(const Slots<T>& S, uint32_t j,
                                            typename std::conditional<is_fp64<T>(), double, float>::type p[3], T u[3],
                                            int32_t& id, int32_t& cell) {
  if constexpr (is_fp64<T>()) {
    const double2 A = ldr<double2, T>(S.a, j), Bv = ldr<double2, T>(S.b, j), C = ldr<double2, T>(S.c, j);
    p[0] = A.x;
    p[1] = A.y;
    p[2] = Bv.x;
    u[0] = Bv.y;
    u[1] = C.x;
    u[2] = C.y;
    id = ld<int32_t>(S.id, j);
    cell = 0;
  } else {
    const float4 A = ldr<float4, T>(S.a, j), Bv = ldr<float4, T>(S.b, j);
    p[0] = A.x;
    p[1] = A.y;
    p[2] = A.z;
    id = __float_as_int(A.w);
    u[0] = Bv.x;
    u[1] = Bv.y;
    u[2] = Bv.z;
    cell = __float_as_int(Bv.w);
  }
}

// Store a packet into slot j of S (FP32: with its home cell; WGT: with its weight).
template <typename T, bool WGT>
__device__ __forceinline__ void store_packet(const Slots<T>& S, uint32_t j, const double x[3], const T f[3],
                                             const T u[3], T wv, int32_t id, int32_t cell) {
  if constexpr (is_fp64<T>()) {
    str<double2, T>(S.a, j, make_double2(x[0], x[1]));
    str<double2, T>(S.b, j, make_double2(x[2], u[0]));
    str<double2, T>(S.c, j, make_double2(u[1], u[2]));
    st<int32_t>(S.id, j, id);
  } else {
    str<float4, T>(S.a, j, make_float4(f[0], f[1], f[2], __int_as_float(id)));
    str<float4, T>(S.b, j, make_float4(u[0], u[1], u[2], __int_as_float(cell)));
  }
  if constexpr (WGT) st<T>(S.w, j, wv);
}

// Load the packet of an inbox or overflow slot (home cell not implied by the slot).
template <typename T, bool WGT>
__device__ __forceinline__ void load_free(const Slots<T>& S, uint32_t j, const RunConsts& k, int home[3], T f[3],
                                          double xa[3], T u[3], T& wv, int32_t& id) {
  using PX = typename std::conditional<is_fp64<T>(), double, float>::type;
  PX p[3];
  int32_t cell;
  load_packet<T>(S, j, p, u, id, cell);
  wv = WGT ? ld<T>(S.w, j) : T(1);
  if constexpr (is_fp64<T>()) {
    const int n3[3] = {k.nx, k.ny, k.nz};
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      xa[d] = p[d];
      const double s = xa[d] * k.inv_dx;
      const double fl = floor(s);
      home[d] = wrapm((int)fl, n3[d]);
      f[d] = s - fl;
    }
  } else {
    cell_coords(cell, k, home);
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      f[d] = p[d];
      xa[d] = 0.0;
    }
  }
}

// Home cell of an inbox packet (FP64 from its position, FP32 from its cell word).
template <typename T>
__device__ __forceinline__ void home_of(const Slots<T>& S, uint32_t j, const RunConsts& k, int h[3]) {
  if constexpr (is_fp64<T>()) {
    const int n3[3] = {k.nx, k.ny, k.nz};
    const double2 A = ldr<double2, T>(S.a, j);
    const double z = ldr<double, T>(S.b, j);
    h[0] = wrapm((int)floor(A.x * k.inv_dx), n3[0]);
    h[1] = wrapm((int)floor(A.y * k.inv_dx), n3[1]);
    h[2] = wrapm((int)floor(z * k.inv_dx), n3[2]);
  } else {
    cell_coords(ldr<int32_t, T>(S.b + 12, j), k, h);
  }
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

// Inbox slot (in the next buffer) for a packet of this workgroup's tile whose new
// (wrapped) home cell is h: the part of h's tile inbox reserved for packets from this
// tile (the self part when h is in this tile).  Returns -1 when the part is full or h's
// tile is not a neighbour (the packet then needs an overflow slot).
__device__ __forceinline__ int place_inbox(const StepView& V, int ttx, int tty, int ttz, int* cntD,
                                           const int* sDcap, const int* sDoff, const int h[3]) {
  const int tx = (int)((unsigned)h[0] / kCellTile), ty = (int)((unsigned)h[1] / kCellTile),
            tz = (int)((unsigned)h[2] / kCellTile);
  const int sx = tile_step(tx, ttx, V.ntx), sy = tile_step(ty, tty, V.nty), sz = tile_step(tz, ttz, V.ntz);
  if (sx > 1 || sy > 1 || sz > 1) return -1;
  const int dir = (sx + 1) + 3 * ((sy + 1) + 3 * (sz + 1));
  const int s = atomicAdd(&cntD[dir], 1);
  if (s < sDcap[dir]) {
    const uint32_t t = (uint32_t)tx + (uint32_t)V.ntx * ((uint32_t)ty + (uint32_t)V.nty * (uint32_t)tz);
    return (int)((uint32_t)V.ib0 + t * (uint32_t)V.per_tile + (uint32_t)(sDoff[dir] + s));
  }
  return -1;
}

// Slot in the return part of the inbox of h's tile, which any workgroup fills through a
// global counter (cleared after every step), or -1 when that part is full.
__device__ __forceinline__ int place_return(const StepView& V, const int h[3]) {
  const uint32_t t = (unsigned)h[0] / kCellTile +
                     (uint32_t)V.ntx * ((unsigned)h[1] / kCellTile + (uint32_t)V.nty * ((unsigned)h[2] / kCellTile));
  const int s = atomicAdd(V.icnt_out + (int64_t)t * kParts + kReturnPart, 1);
  if (s < V.dcap[kReturnPart])
    return (int)((uint32_t)V.ib0 + t * (uint32_t)V.per_tile + (uint32_t)(V.doff[kReturnPart] + s));
  return -1;
}

// Slot in the next overflow list (global counter), or -1 and ERR_TILE when that is
// full too (the packet is then lost and the step reports it).
__device__ __forceinline__ int place_overflow(const StepView& V, uint32_t& err) {
  const int s = atomicAdd(V.icnt_out + V.ntiles * kParts, 1);
  if ((int64_t)s < V.ocap) return (int)((uint32_t)V.ov0 + (uint32_t)s);
  err |= ERR_TILE;
  return -1;
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
    // periodic wrap and the cell index, each in a branch that only the lanes leaving
    // the box (or landing on its upper face by rounding) take: a wave without such a
    // lane skips it
    bool out = false;
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      const double stp = s * un[d];
      bad |= fabs(stp) > k.max_step * k.dx;
      const double y = xa[d] + stp;
      out |= !(y >= 0.0 && y < L3[d]);
      xn[d] = y;
      fn[d] = 0;
    }
    if (out) {
      #pragma unroll
      for (int d = 0; d < 3; ++d) xn[d] = wrap_coord(xn[d], L3[d]);
    }
    bool hout = false;
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      h[d] = (int)floor(xn[d] * k.inv_dx);
      hout |= (unsigned)h[d] >= (unsigned)n3[d];
    }
    if (hout) {
      #pragma unroll
      for (int d = 0; d < 3; ++d) h[d] = wrap_near(h[d], n3[d]);
    }
  } else {
    bool hout = false;
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      const float stp = s * un[d];
      bad |= fabsf(stp) > (float)k.max_step;
      float fo = f[d] + stp;
      const float fl = floorf(fo);
      int hd = home[d] + (int)fl;
      fo -= fl;
      if (fo >= 1.0f) {
        fo = 0.0f;
        hd += 1;
      }
      h[d] = hd;
      hout |= (unsigned)hd >= (unsigned)n3[d];
      fn[d] = fo;
      xn[d] = 0.0;
    }
    // the periodic wrap of the cell index, in a branch only lanes leaving the box take
    if (hout) {
      #pragma unroll
      for (int d = 0; d < 3; ++d) h[d] = wrap_near(h[d], n3[d]);
    }
  }
  if (!bad) return 0u;
  return fin ? (uint32_t)ERR_COURANT : (uint32_t)ERR_NAN;
}

// Weight modes of the step: packets without weights, with weights (per-packet mass
// M_j = mass * w_j), and with weights that decay under catastrophic losses.  FP64
// without losses runs two workgroups per CU (two waves per SIMD, 256 registers; with
// losses that bound spills) and FP32 three by its register count.
constexpr int kNoWeights = 0;
constexpr int kWeights = 1;
constexpr int kLosses = 2;
template <typename T, int WM>
constexpr bool two_wave_step() {
  return is_fp64<T>() && WM != kLosses;
}

// LDS of the quad loop (per-wave exchange areas) and of the workgroup's tail
// (exchange accumulator of the tile plus halo), which share the same bytes.
template <typename T>
struct LoopLds {
  T Pk[kThreads / 64][16 * kPkQuad<T>];  // per lane: the packet's weights, offsets and exchange values
  T Rs[kThreads / 64][64 * kRsStride];    // per lane: its partial field sums
};
struct TailLds {
  double Acc[4][kAccPitch];
};
template <typename T>
union StepLds {
  LoopLds<T> loop;
  TailLds tail;
};

// One step of the packets of one tile.  M: 2 (CIC) or 3 (TSC); DEP: deposit the
// exchange; WM: weight mode; PUSH: the momentum update (Boris, Vay or Higuera-Cary).
template <int M, typename T, bool DEP, int WM, int PUSH>
__global__ void __launch_bounds__(kThreads, (two_wave_step<T, WM>() ? 2 : 1))
    cells_step_kernel(StepView V, const T* __restrict__ E, const T* __restrict__ B, const T* __restrict__ NN,
                      double* __restrict__ dM, double* __restrict__ dE, RunConsts k) {
  constexpr bool LOSS = WM == kLosses;
  constexpr bool WGT = WM != kNoWeights;
  constexpr int NF = LOSS ? 7 : 6;
  using PX = typename std::conditional<is_fp64<T>(), double, float>::type;  // position or offset
  __shared__ T Fs[NF][kRegionCells];
  __shared__ __attribute__((aligned(16))) StepLds<T> U;
  __shared__ int cntD[kDirs];      // inbox slots this workgroup took, by direction
  __shared__ int sDcap[kParts];
  __shared__ int sDoff[kParts + 1];
  __shared__ int sPre[kParts + 1];  // prefix of this tile's inbox counts by part
  __shared__ int qCnt[kCellTileCells];   // listed inbox packets per local cell
  __shared__ int qOff[kCellTileCells];   // their prefix
  __shared__ int qFill[kCellTileCells];
  __shared__ int sNb[kCellTileCells];    // bucket packets per local cell
  __shared__ int sPerm[kCellTileCells];  // local cell of each quad, fullest first
  __shared__ uint32_t sQ[kQueue];        // inbox slot of each listed packet, grouped by cell
  __shared__ unsigned char sLc[kQueue];  // local cell of each listed packet, in inbox order

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
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const uint32_t cap = (uint32_t)V.cap;
  uint32_t err = 0;
  const Slots<T> Si = slots_of<T>(V.in);
  const Slots<T> So = slots_of<T>(V.out);

  // ------------------------------------------------------------ prologue
  // bucket counts of the tile's cells (one per lane of the first wave), inbox counts by
  // direction, and the fields of the tile plus a one-cell halo
  bool lvalid = false;
  int nb_l = 0;
  if (tid < kCellTileCells) {
    const int gx = ttx * kCellTile + (tid & 3), gy = tty * kCellTile + ((tid >> 2) & 3),
              gz = ttz * kCellTile + (tid >> 4);
    lvalid = gx < k.nx && gy < k.ny && gz < k.nz;
    if (lvalid) {
      const int v = V.bcnt_in[gx + (int64_t)k.nx * (gy + (int64_t)k.ny * gz)];
      nb_l = v < (int)cap ? v : (int)cap;
    }
  }
  const int cin = tid < kParts ? V.icnt_in[(int64_t)tile * kParts + tid] : 0;
  for (int r = tid; r < kRegionCells; r += kThreads) {
    const int rx = r % kRegionEdge, ry = (r / kRegionEdge) % kRegionEdge, rz = r / (kRegionEdge * kRegionEdge);
    const int64_t rc =
        wrapm(ox + rx, k.nx) + (int64_t)k.nx * (wrapm(oy + ry, k.ny) + (int64_t)k.ny * wrapm(oz + rz, k.nz));
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      Fs[d][r] = E[d * nc + rc];
      Fs[3 + d][r] = B[d * nc + rc];
    }
    if constexpr (LOSS) Fs[6][r] = NN[rc];
  }
  if (tid < kCellTileCells) {
    qCnt[tid] = 0;
    qFill[tid] = 0;
    sNb[tid] = nb_l;
    // part capacities and offsets by lane (uniform kernel-argument reads), then the
    // prefix of the clamped inbox counts across the first wave
    int dcap = 0, doff = V.doff[kParts];
    #pragma unroll
    for (int d = 0; d < kParts; ++d) {
      dcap = tid == d ? V.dcap[d] : dcap;
      doff = tid == d ? V.doff[d] : doff;
    }
    if (tid < kDirs) cntD[tid] = 0;
    if (tid < kParts) sDcap[tid] = dcap;
    if (tid <= kParts) sDoff[tid] = doff;
    const int c = cin < dcap ? cin : dcap;
    int incl = c;
    #pragma unroll
    for (int o = 1; o < 32; o <<= 1) {
      const int y = __shfl_up(incl, o);
      if (lane >= o) incl += y;
    }
    if (tid <= kParts) sPre[tid] = incl - c;
  }
  __syncthreads();

  // the tile's inbox packets: the first kQueue are listed by cell in LDS and join the
  // quad loop after their cell's bucket; further ones take the per-packet path
  const int nin = sPre[kParts];
  const int nlist = nin < kQueue ? nin : kQueue;
  const uint32_t ibase = (uint32_t)(V.ib0 + (int64_t)tile * V.per_tile);
  auto inbox_slot = [&](int i) -> uint32_t {
    int dir = 0;
    #pragma unroll
    for (int d = 1; d < kParts; ++d) dir += (i >= sPre[d]) ? 1 : 0;
    return ibase + (uint32_t)(sDoff[dir] + (i - sPre[dir]));
  };
  // local cell of a home cell of this tile (anything else is a filing error: flagged,
  // and the packet is taken by the nearest cell of the tile)
  auto local_of = [&](const int h[3]) -> int {
    int l[3] = {h[0] - ttx * kCellTile, h[1] - tty * kCellTile, h[2] - ttz * kCellTile};
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      if (l[d] < 0 || l[d] >= kCellTile) err |= ERR_TILE;
      l[d] = min(max(l[d], 0), kCellTile - 1);
    }
    return l[0] + kCellTile * (l[1] + kCellTile * l[2]);
  };
  for (int i = tid; i < nlist; i += kThreads) {
    int h[3];
    home_of<T>(Si, inbox_slot(i), k, h);
    const int lc = local_of(h);
    sLc[i] = (unsigned char)lc;
    atomicAdd(&qCnt[lc], 1);
  }
  __syncthreads();
  if (tid < kCellTileCells) {
    // prefix of the listed counts, and the quads' cells in order of total count (fullest
    // first, ties by cell index), so that the cells of a wave need similar round counts
    const int c = qCnt[tid];
    int incl = c;
    #pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int y = __shfl_up(incl, o);
      if (lane >= o) incl += y;
    }
    qOff[tid] = incl - c;
    const int n_l = lvalid ? nb_l + c : -1;
    int rank = 0;
    #pragma unroll
    for (int m = 0; m < kCellTileCells; ++m) {
      const int nm = __builtin_amdgcn_readlane(n_l, m);
      rank += (nm > n_l || (nm == n_l && m < tid)) ? 1 : 0;
    }
    sPerm[rank] = tid;
  }
  __syncthreads();
  for (int i = tid; i < nlist; i += kThreads) {
    const int lc = sLc[i];
    sQ[qOff[lc] + atomicAdd(&qFill[lc], 1)] = inbox_slot(i);
  }
  __syncthreads();

  const T h = (T)k.h, hb = (T)k.hb;
  const T pf = (T)k.pfac, ef = (T)k.efac;
  const T lrate = (T)k.lrate;

  // ------------------------------------------------------------ quads: one cell each
  const int q = tid & 3;
  const int quad = tid >> 2;
  const int qbase = lane & ~3;  // first lane of this quad within the wave
  const int lc = sPerm[quad];
  const int lx = lc & 3, ly = (lc >> 2) & 3, lz = lc >> 4;
  const int home[3] = {ttx * kCellTile + lx, tty * kCellTile + ly, ttz * kCellTile + lz};
  const bool valid = home[0] < k.nx && home[1] < k.ny && home[2] < k.nz;
  const int nb = sNb[lc];
  const int nq = valid ? qCnt[lc] : 0;
  const int qo = qOff[lc];
  const int n = nb + nq;
  T* pkw = &U.loop.Pk[tid >> 6][0];
  T* rsw = &U.loop.Rs[tid >> 6][0];

  // this lane's field components on the 27 nodes around the cell.  Without losses the
  // quad holds E_x, E_y, E_z, B_x in F0 (lane q: component q) and B_y, B_z, B_y, B_z in
  // F1, so the six components of its four packets take six passes: four over F0 and two
  // over F1, where lanes 0, 1 serve packets 0, 2 and lanes 2, 3 packets 1, 3.  With
  // losses lane q < 3 holds E_q, B_q and lane 3 the nucleon density.  With TSC the node
  // values are turned into the interpolant's coefficients once (tsc_coefficients) and
  // each pass evaluates them at a packet's three offsets.
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

  // packet state of the next round (loaded a round ahead; the other waves of the SIMD
  // cover the latency): packet kk of the cell is slot kk of its bucket for kk < nb, then
  // its listed inbox packets
  T pu[3] = {T(0), T(0), T(0)};
  PX px[3] = {PX(0), PX(0), PX(0)};
  int32_t pid = 0;
  T pw = T(1);
  auto fetch = [&](int rd) {
    const int kk = 4 * rd + q;
    if (kk < n) {
      const int qi = min(max(qo + kk - nb, 0), kQueue - 1);
      const uint32_t j = kk < nb ? slot32((uint32_t)tile, (uint32_t)kk, (uint32_t)lc, cap) : sQ[qi];
      int32_t cell_unused;
      load_packet<T>(Si, j, px, pu, pid, cell_unused);
      if constexpr (WGT) pw = ld<T>(Si.w, j);
    }
  };
  fetch(0);

  // the stayers' stream of this cell in the next buffer
  int S = 0;
  // the previous round's packet, stored at the start of the next round (just before
  // that round's prefetch) so that the loop never waits on its own fresh stores
  uint32_t oj = 0;
  bool ost = false;
  double oxn[3] = {0.0, 0.0, 0.0};
  T ofn[3] = {T(0), T(0), T(0)}, oun[3] = {T(0), T(0), T(0)};
  T ow = T(1);
  int32_t oid = 0, ocell = 0;
  auto flush = [&]() {
    if (ost) store_packet<T, WGT>(So, oj, oxn, ofn, oun, ow, oid, ocell);
  };
  auto round = [&](const int rd) {
    // A lane past its cell's count computes on the registers of its last packet (or the
    // zeros they start with): finite values whose results are dropped, its exchange
    // values being scaled by zero and its packet not stored.
    const bool act = 4 * rd + q < n;
    T f[3], u[3];
    double xa[3] = {0.0, 0.0, 0.0};
    const int32_t id = pid;
    const T wv = pw;
    const T pfa = act ? pf : T(0), efa = act ? ef : T(0);
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      if constexpr (is_fp64<T>()) {
        xa[d] = px[d];
        const double s = xa[d] * k.inv_dx;
        f[d] = s - floor(s);
      } else {
        f[d] = (T)px[d];
      }
      u[d] = pu[d];
    }
    flush();
    fetch(rd + 1);

    // own weights -> LDS: x weights, then the nine y-z products
    {
      T wx[3], wy[3], wz[3];
      weights3<M, T>(f[0], wx);
      weights3<M, T>(f[1], wy);
      weights3<M, T>(f[2], wz);
      T* o = pkw + pk_at<T>(lane);
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
        const T* wj = pkw + pk_at<T>(qbase + J);
        if constexpr (M == 3) {
          const T dv[3] = {wj[12], wj[13], wj[14]};
          rsw[lane * kRsStride + 2 * J] = tsc_poly<T>(dv, F0);
          rsw[lane * kRsStride + 2 * J + 1] = tsc_poly<T>(dv, F1);
        } else {
          T w[12];
          #pragma unroll
          for (int i = 0; i < 12; ++i) w[i] = wj[i];
          rsw[lane * kRsStride + 2 * J] = stencil_sum<T>(w, F0);
          rsw[lane * kRsStride + 2 * J + 1] = stencil_sum<T>(w, F1);
        }
      }
      wave_sync();
      #pragma unroll
      for (int c = 0; c < 3; ++c) {
        eb[c] = rsw[(qbase + c) * kRsStride + 2 * q];
        eb[3 + c] = rsw[(qbase + c) * kRsStride + 2 * q + 1];
      }
    } else {
      #pragma unroll
      for (int J = 0; J < 4; ++J) {
        const T* wj = pkw + pk_at<T>(qbase + J);
        if constexpr (M == 3) {
          const T dv[3] = {wj[12], wj[13], wj[14]};
          rsw[lane * kRsStride + J] = tsc_poly<T>(dv, F0);
        } else {
          T w[12];
          #pragma unroll
          for (int i = 0; i < 12; ++i) w[i] = wj[i];
          rsw[lane * kRsStride + J] = stencil_sum<T>(w, F0);
        }
      }
      #pragma unroll
      for (int p = 0; p < 2; ++p) {
        const T* wj = pkw + pk_at<T>(qbase + 2 * p + (q >> 1));
        if constexpr (M == 3) {
          const T dv[3] = {wj[12], wj[13], wj[14]};
          rsw[lane * kRsStride + 4 + p] = tsc_poly<T>(dv, F1);
        } else {
          T w[12];
          #pragma unroll
          for (int i = 0; i < 12; ++i) w[i] = wj[i];
          rsw[lane * kRsStride + 4 + p] = stencil_sum<T>(w, F1);
        }
      }
      wave_sync();
      #pragma unroll
      for (int c = 0; c < 4; ++c) eb[c] = rsw[(qbase + c) * kRsStride + q];
      const int hy = qbase + 2 * (q & 1);  // lane holding B_y for this lane's packet
      eb[4] = rsw[hy * kRsStride + 4 + (q >> 1)];
      eb[5] = rsw[(hy + 1) * kRsStride + 4 + (q >> 1)];
    }

    // kick (Eq. (11))
    const Kick<T> kq = kick<PUSH, T>(u[0], u[1], u[2], eb[0], eb[1], eb[2], eb[3], eb[4], eb[5], h, hb);
    const T un[3] = {u[0] + kq.dux, u[1] + kq.duy, u[2] + kq.duz};
    // losses: weight update; the exchange becomes the change of the weighted totals,
    // wn du - w lost u (momentum) and wn dgamma - w lost gamma (energy)
    T wn = wv, lost = T(0);
    if constexpr (LOSS) {
      const T nnp = rsw[(qbase + 3) * kRsStride + 2 * q];
      loss_step<T>(un[0], un[1], un[2], nnp, lrate, wv, &wn, &lost);
    }

    // exchange (Eq. (12)) into the quad's registers, lane q taking component q
    if constexpr (DEP) {
      T* o = pkw + pk_at<T>(lane);
      if constexpr (LOSS) {
        const T wl = wv * lost;
        o[12] = pfa * (wn * kq.dux - wl * u[0]);
        o[13] = pfa * (wn * kq.duy - wl * u[1]);
        o[14] = pfa * (wn * kq.duz - wl * u[2]);
        o[15] = efa * (wn * kq.dg - wl * kq.g0);
      } else if constexpr (WGT) {
        o[12] = pfa * (wv * kq.dux);
        o[13] = pfa * (wv * kq.duy);
        o[14] = pfa * (wv * kq.duz);
        o[15] = efa * (wv * kq.dg);
      } else {
        o[12] = pfa * kq.dux;
        o[13] = pfa * kq.duy;
        o[14] = pfa * kq.duz;
        o[15] = efa * kq.dg;
      }
      wave_sync();
      #pragma unroll
      for (int J = 0; J < 4; ++J) {
        const T* wj = pkw + pk_at<T>(qbase + J);
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
      // past the drift and the placement, keeping the 52 values read above live
      // across them (FP64 357 registers and one wave per SIMD, FP32 209 and two)
      #pragma unroll
      for (int i = 0; i < 27; ++i) asm volatile("" : "+v"(D[i]));
    }
    wave_sync();

    // drift; a packet still in its cell goes to the next slot of the cell's stream
    // (its rank among the quad's stayers of this round), any other to an inbox part
    int hn[3];
    const uint32_t e1 = drift3<T>(k, home, f, xa, un, hn, oxn, ofn);
    err |= act ? e1 : 0u;
    const bool stay = act && hn[0] == home[0] && hn[1] == home[1] && hn[2] == home[2];
    const uint32_t qm = (uint32_t)(__ballot(stay) >> qbase) & 0xFu;
    const int slot = S + __popc(qm & ((1u << q) - 1u));
    S += __popc(qm);
    ost = act;
    if (stay && slot < (int)cap) {
      oj = slot32((uint32_t)tile, (uint32_t)slot, (uint32_t)lc, cap);
    } else if (act) {
      int j2 = place_inbox(V, ttx, tty, ttz, cntD, sDcap, sDoff, hn);
      if (j2 < 0) j2 = place_return(V, hn);
      if (j2 < 0) j2 = place_overflow(V, err);
      ost = j2 >= 0;
      oj = (uint32_t)j2;
    }
    #pragma unroll
    for (int d = 0; d < 3; ++d) oun[d] = un[d];
    ow = wn;
    oid = id;
    ocell = hn[0] + k.nx * (hn[1] + k.ny * hn[2]);
  };
  // two rounds per iteration: the loop-carried registers (deposit accumulators, the
  // prefetched packet) then keep their places instead of being copied every round
  const int rounds = (n + 3) >> 2;
  for (int rd = 0; __ballot(rd < rounds) != 0; rd += 2) {
    round(rd);
    if (__ballot(rd + 1 < rounds) == 0) break;
    round(rd + 1);
  }
  flush();

  // ------------------------------------------------------------ tail
  __syncthreads();  // every wave is out of its quad loop: the exchange areas become the accumulator
  double* acc = &U.tail.Acc[0][0];
  if constexpr (DEP) {
    for (int r = tid; r < 4 * kAccPitch; r += kThreads) acc[r] = 0.0;
    __syncthreads();
    if (n > 0) {
      #pragma unroll
      for (int c = 0; c < 3; ++c)
        #pragma unroll
        for (int b = 0; b < 3; ++b)
          #pragma unroll
          for (int a = 0; a < 3; ++a) {
            const int r = (lx + a) + kRegionEdge * ((ly + b) + kRegionEdge * (lz + c));
            atomicAdd(&acc[q * kAccPitch + r], (double)D[a + 3 * (b + 3 * c)]);
          }
    }
  }

  // one packet per thread: gather from the staged fields, deposit with LDS atomics, and
  // the next buffer's inbox (never a bucket: the cells' streams are closed)
  auto process = [&](const int hm[3], const T f[3], const double xa[3], const T u[3], T wv, int32_t id) {
    // region coordinates of node home-1 (these packets all live in this tile; the
    // clamp only keeps a misfiled packet, already flagged, inside the staged region)
    const int bx = min(max(hm[0] - ttx * kCellTile, 0), kCellTile - 1);
    const int by = min(max(hm[1] - tty * kCellTile, 0), kCellTile - 1);
    const int bz = min(max(hm[2] - ttz * kCellTile, 0), kCellTile - 1);
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
    if constexpr (DEP) {
      const T wl = wv * lost;
      const T qv[4] = {pf * (wn * kq.dux - wl * u[0]), pf * (wn * kq.duy - wl * u[1]),
                       pf * (wn * kq.duz - wl * u[2]), ef * (wn * kq.dg - wl * kq.g0)};
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
              for (int d = 0; d < 4; ++d) atomicAdd(&acc[d * kAccPitch + r], (double)(W * qv[d]));
            }
          }
        }
    }
    int hn[3];
    double xn[3];
    T fn[3];
    err |= drift3<T>(k, hm, f, xa, un, hn, xn, fn);
    int j2 = place_inbox(V, ttx, tty, ttz, cntD, sDcap, sDoff, hn);
    if (j2 < 0) j2 = place_return(V, hn);
    if (j2 < 0) j2 = place_overflow(V, err);
    if (j2 >= 0)
      store_packet<T, WGT>(So, (uint32_t)j2, xn, fn, un, wn, id, hn[0] + k.nx * (hn[1] + k.ny * hn[2]));
  };
  for (int i = kQueue + tid; i < nin; i += kThreads) {
    int hm[3];
    T f[3], u[3];
    double xa[3];
    int32_t id;
    T wv;
    load_free<T, WGT>(Si, inbox_slot(i), k, hm, f, xa, u, wv, id);
    (void)local_of(hm);
    process(hm, f, xa, u, wv, id);
  }

  // ------------------------------------------------------------ overflow list, shared by all workgroups
  {
    int nov = V.icnt_in[ntiles * kParts];
    nov = (int64_t)nov < V.ocap ? nov : (int)V.ocap;
    const int n3[3] = {k.nx, k.ny, k.nz};
    for (int64_t i = (int64_t)blockIdx.x * kThreads + tid; i < nov; i += (int64_t)gridDim.x * kThreads) {
      int hm[3];
      T f[3], u[3];
      double xa[3];
      int32_t id;
      T wv;
      load_free<T, WGT>(Si, (uint32_t)(V.ov0 + i), k, hm, f, xa, u, wv, id);
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
            nodes[a + 3 * (b + 3 * c)] = wrapm(hm[0] - 1 + a, n3[0]) +
                (int64_t)k.nx * (wrapm(hm[1] - 1 + b, n3[1]) + (int64_t)k.ny * wrapm(hm[2] - 1 + c, n3[2]));
      T eb[NF];
      gather27<NF, T>(w, [&](int node, int d) {
        return d < 3 ? E[d * nc + nodes[node]] : (d < 6 ? B[(d - 3) * nc + nodes[node]] : NN[nodes[node]]);
      }, eb);
      const Kick<T> kq = kick<PUSH, T>(u[0], u[1], u[2], eb[0], eb[1], eb[2], eb[3], eb[4], eb[5], h, hb);
      const T un[3] = {u[0] + kq.dux, u[1] + kq.duy, u[2] + kq.duz};
      T wn = wv, lost = T(0);
      if constexpr (LOSS) loss_step<T>(un[0], un[1], un[2], eb[NF - 1], lrate, wv, &wn, &lost);
      if constexpr (DEP) {
        const T wl = wv * lost;
        const T qv[4] = {pf * (wn * kq.dux - wl * u[0]), pf * (wn * kq.duy - wl * u[1]),
                         pf * (wn * kq.duz - wl * u[2]), ef * (wn * kq.dg - wl * kq.g0)};
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
      err |= drift3<T>(k, hm, f, xa, un, hn, xn, fn);
      int j2 = place_return(V, hn);
      if (j2 < 0) j2 = place_overflow(V, err);
      if (j2 >= 0)
        store_packet<T, WGT>(So, (uint32_t)j2, xn, fn, un, wn, id, hn[0] + k.nx * (hn[1] + k.ny * hn[2]));
    }
  }
  if (err) set_status(k.status, err);
  __syncthreads();

  // ------------------------------------------------------------ outputs
  if constexpr (DEP) {
    double* out = V.halo + (int64_t)tile * 4 * kRegionCells;
    for (int i = tid; i < 4 * kRegionCells; i += kThreads) {
      const int d = i / kRegionCells;
      const double v = acc[d * kAccPitch + (i - d * kRegionCells)];
      out[i] = V.accumulate ? out[i] + v : v;
    }
  }
  if (q == 0 && valid) V.bcnt_out[home[0] + (int64_t)k.nx * (home[1] + (int64_t)k.ny * home[2])] = S < (int)cap ? S : (int)cap;
  if (tid >= 64 && tid < 64 + kDirs) {
    // count of part `dir` of the inbox of the tile at offset dir; this workgroup is
    // that part's only writer
    const int dir = tid - 64;
    const int sx = dir % 3 - 1, sy = (dir / 3) % 3 - 1, sz = dir / 9 - 1;
    const int64_t t = wrapm(ttx + sx, V.ntx) +
                      (int64_t)V.ntx * (wrapm(tty + sy, V.nty) + (int64_t)V.nty * wrapm(ttz + sz, V.ntz));
    const int v = cntD[dir];
    V.icnt_out[t * kParts + dir] = v < sDcap[dir] ? v : sDcap[dir];
  }
}

// After a step (or the last step of a call): add the per-tile exchange accumulators
// into the grid (a cell takes every region slot, of its own tile and of neighbouring
// tiles' halos, that maps onto it), and clear the counters of the buffer the step
// consumed that packets take with global atomics.  In a coupled step dM, dE are the gas
// momentum and energy, and the cell's E is refreshed from the updated momentum.  With
// dM NULL only the counters are cleared.
__global__ void cells_post_kernel(StepView V, double* dM, double* dE, GasLink gas, RunConsts k) {
  const int64_t nc = k.ncells;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  // the consumed buffer takes the next step's output: clear its counters that packets
  // take with global atomics (the overflow list and the tiles' return parts)
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid == 0) V.icnt_in[V.ntiles * kParts] = 0;
  for (int64_t t = gid; t < V.ntiles; t += stride) V.icnt_in[t * kParts + kReturnPart] = 0;
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
  const Slots<T> So = slots_of<T>(L.buf[0]);
  const bool wgt = P.w && L.buf[0].w;
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
    int64_t j;
    if (slot < L.cap) {
      j = bucket_index(h, slot, L.ntx, L.nty, L.cap);
    } else {
      const int64_t t = h[0] / kCellTile + (int64_t)L.ntx * (h[1] / kCellTile + (int64_t)L.nty * (h[2] / kCellTile));
      const int is = atomicAdd(&L.icnt[0][t * kParts + kSelfDir], 1);
      const int ir = is < L.dcap[kSelfDir] ? 0 : atomicAdd(&L.icnt[0][t * kParts + kReturnPart], 1);
      if (is < L.dcap[kSelfDir]) {
        j = L.ib0 + t * L.per_tile + L.doff[kSelfDir] + is;
      } else if (ir < L.dcap[kReturnPart]) {
        j = L.ib0 + t * L.per_tile + L.doff[kReturnPart] + ir;
      } else {
        const int os = atomicAdd(&L.icnt[0][L.ntiles * kParts], 1);
        if ((int64_t)os >= L.ocap) {
          set_status(k.status, ERR_TILE);
          continue;
        }
        j = L.ov0 + os;
      }
    }
    const T wv = wgt ? P.w[i] : T(1);
    if (wgt) store_packet<T, true>(So, (uint32_t)j, x, f, u, wv, id, key);
    else store_packet<T, false>(So, (uint32_t)j, x, f, u, wv, id, key);
  }
}

// Clamped occupancy of every store, in compaction order: cells, tile directions, overflow.
__global__ void cells_counts_kernel(CellLists L, int64_t nc, int32_t* __restrict__ out) {
  const int cur = L.cur;
  const int64_t ni = L.ntiles * kParts;
  const int64_t n = nc + ni + 1;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    int v, cap;
    if (i < nc) {
      v = L.bcnt[cur][i];
      cap = L.cap;
    } else if (i < nc + ni) {
      v = L.icnt[cur][i - nc];
      const int dir = (int)((i - nc) % kParts);
      cap = 0;
      #pragma unroll
      for (int d = 0; d < kParts; ++d) cap = (dir == d) ? L.dcap[d] : cap;
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
  using PX = typename std::conditional<is_fp64<T>(), double, float>::type;
  const Slots<T> Q = slots_of<T>(S);
  PX p[3];
  T u[3];
  int32_t id, rec_cell;
  load_packet<T>(Q, (uint32_t)j, p, u, id, rec_cell);
  #pragma unroll
  for (int d = 0; d < 3; ++d) {
    if constexpr (is_fp64<T>()) P.x[d * P.np + o] = p[d];
    else P.off[d * P.np + o] = p[d];
    P.u[d * P.np + o] = u[d];
  }
  if constexpr (!is_fp64<T>()) P.cell[o] = cell < 0 ? rec_cell : cell;
  P.id[o] = id;
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
  for (int sl = lane; sl < n; sl += 64)
    copy_out<T>(P, S, (int64_t)slot32((uint32_t)t, (uint32_t)sl, (uint32_t)lc, (uint32_t)L.cap), offs[c] + sl,
                (int32_t)c);
}

// The inbox parts of buffer cur -> caller arrays, one workgroup per tile: the tile's
// parts are consecutive in the prefix sum, so its packets fill one contiguous range.
template <typename T>
__global__ void __launch_bounds__(kThreads) cells_compact_parts_kernel(Packets<T> P, CellLists L,
                                                                        const int32_t* __restrict__ offs, RunConsts k) {
  __shared__ int pre[kParts + 1];
  const SlotArrays& S = L.buf[L.cur];
  const int64_t nc = k.ncells;
  const int64_t t = blockIdx.x;
  const int64_t e0 = nc + t * kParts;
  if (threadIdx.x < 64) {
    const int c = threadIdx.x < kParts ? offs[e0 + threadIdx.x + 1] - offs[e0 + threadIdx.x] : 0;
    int incl = c;
    #pragma unroll
    for (int o = 1; o < 32; o <<= 1) {
      const int y = __shfl_up(incl, o);
      if ((int)(threadIdx.x & 63) >= o) incl += y;
    }
    if (threadIdx.x <= kParts) pre[threadIdx.x] = incl - c;
  }
  __syncthreads();
  const int tot = pre[kParts];
  const int64_t o0 = offs[e0];
  for (int i = threadIdx.x; i < tot; i += kThreads) {
    int dir = 0;
    #pragma unroll
    for (int d = 1; d < kParts; ++d) dir += (i >= pre[d]) ? 1 : 0;
    const int64_t s = L.ib0 + t * L.per_tile + L.doff[dir] + (i - pre[dir]);
    copy_out<T>(P, S, s, o0 + i, -1);
  }
}

// The overflow list of buffer cur -> caller arrays at its prefix-sum offset.
template <typename T>
__global__ void cells_compact_overflow_kernel(Packets<T> P, CellLists L, const int32_t* __restrict__ offs,
                                              RunConsts k) {
  const SlotArrays& S = L.buf[L.cur];
  const int64_t obase = (int64_t)k.ncells + L.ntiles * kParts;
  const int64_t n = offs[obase + 1] - offs[obase];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    copy_out<T>(P, S, L.ov0 + i, offs[obase] + i, -1);
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

SlotArrays carve_slots(Carver& cv, int64_t nslots, bool f32, bool weights) {
  SlotArrays S;
  S.stride = nslots;
  const size_t n = (size_t)nslots;
  char* rec = cv.take((f32 ? 32 : 48) * n);
  S.a = (void*)rec;
  S.b = (void*)(rec + 16);
  S.c = f32 ? nullptr : (void*)(rec + 32);
  S.id = f32 ? nullptr : (int32_t*)cv.take(n * sizeof(int32_t));
  S.w = weights ? (void*)cv.take(n * (f32 ? sizeof(float) : sizeof(double))) : nullptr;
  return S;
}

CellLists carve(int nx, int ny, int nz, int64_t np, int precision, bool weights, uintptr_t base, size_t* bytes,
                int64_t* slots_out) {
  CellLists L;
  const int64_t ncells = (int64_t)nx * ny * nz;
  L.ntx = (nx + kCellTile - 1) / kCellTile;
  L.nty = (ny + kCellTile - 1) / kCellTile;
  L.ntz = (nz + kCellTile - 1) / kCellTile;
  L.ntiles = (int64_t)L.ntx * L.nty * L.ntz;
  // a cell holds Poisson-like counts around the mean: the mean plus four standard
  // deviations and a margin keeps bucket overflow rare (full buckets spill into the
  // tile's self part).  Inbox parts by the number of tile faces crossed: the self part
  // takes the packets that move between the tile's cells (about a tenth of them per
  // step at the Courant limit) and full buckets, eight buckets' worth; faces two; edges
  // half a bucket and corners an eighth, plus margins.  The overflow list takes an
  // eighth of the packets; beyond that a step reports ERR_TILE.
  const int64_t mean = (np + ncells - 1) / ncells;
  const int64_t sd4 = (int64_t)ceil(4.0 * sqrt((double)mean));
  L.cap = (int)((mean + sd4 + 16 + kSlotGroup - 1) / kSlotGroup * kSlotGroup);
  int off = 0;
  for (int d = 0; d < kDirs; ++d) {
    const int axes = (d % 3 != 1) + ((d / 3) % 3 != 1) + (d / 9 != 1);
    const int c = axes == 0 ? 8 * L.cap : axes == 1 ? 2 * L.cap : axes == 2 ? L.cap / 2 + 8 : L.cap / 8 + 8;
    L.dcap[d] = c;
    L.doff[d] = off;
    off += c;
  }
  L.dcap[kReturnPart] = 2 * L.cap + 16;
  L.doff[kReturnPart] = off;
  off += L.dcap[kReturnPart];
  L.doff[kParts] = off;
  L.per_tile = off;
  L.ocap = np / 8 + 4096;
  const bool f32 = precision == 1;
  Carver cv{(base + 255) / 256 * 256};
  const uintptr_t start = cv.p;
  L.ib0 = L.ntiles * L.cap * kCellTileCells;
  L.ov0 = L.ib0 + L.ntiles * L.per_tile;
  L.tr0 = L.ov0 + L.ocap;
  const int64_t slots = L.tr0;
  if (slots_out) *slots_out = slots;
  for (int b = 0; b < 2; ++b) {
    L.buf[b] = carve_slots(cv, slots, f32, weights);
    L.bcnt[b] = (int32_t*)cv.take((size_t)ncells * sizeof(int32_t));
    L.icnt[b] = (int32_t*)cv.take((size_t)(L.ntiles * kParts + 1) * sizeof(int32_t));
  }
  L.halo = (double*)cv.take((size_t)L.ntiles * 4 * kRegionCells * sizeof(double));
  const int64_t nscan = ncells + L.ntiles * kParts + 1;
  // counts (nscan), offsets (nscan + 1), scan temporaries
  L.scan = (int32_t*)cv.take((size_t)(2 * nscan + 1 + (int64_t)exclusive_scan_tmp_ints(nscan)) * sizeof(int32_t));
  L.cur = 0;
  if (bytes) *bytes = (size_t)(cv.p - start) + 256;
  return L;
}

}  // namespace

size_t cell_list_bytes(int nx, int ny, int nz, int64_t np, int precision, bool weights) {
  size_t bytes = 0;
  (void)carve(nx, ny, nz, np, precision, weights, 0, &bytes, nullptr);
  return bytes;
}

bool cell_list_fits(int nx, int ny, int nz, int64_t np, int precision) {
  int64_t slots = 0;
  (void)carve(nx, ny, nz, np, precision, false, 0, nullptr, &slots);
  // the id and weight arrays of a slot store (up to 8 bytes per slot) are addressed by
  // 32-bit byte offsets, the records by 64-bit ones
  (void)precision;
  return slots * 8 < ((int64_t)1 << 32);
}

CellLists cell_list_carve(int nx, int ny, int nz, int64_t np, int precision, bool weights, char* base) {
  return carve(nx, ny, nz, np, precision, weights, (uintptr_t)base, nullptr, nullptr);
}

int64_t cell_list_scan_entries(int nx, int ny, int nz) {
  const int64_t nt = (int64_t)((nx + kCellTile - 1) / kCellTile) * ((ny + kCellTile - 1) / kCellTile) *
                     ((nz + kCellTile - 1) / kCellTile);
  return (int64_t)nx * ny * nz + nt * kParts + 1;
}

template <typename T>
hipError_t launch_cells_build(const Packets<T>& P, CellLists& L, const RunConsts& k, hipStream_t s) {
  L.cur = 0;
  const int64_t ni = L.ntiles * kParts + 1;
  hipLaunchKernelGGL(zero_i32, dim3(grid_for(k.ncells)), dim3(kThreads), 0, s, L.bcnt[0], (int64_t)k.ncells);
  hipLaunchKernelGGL(zero_i32, dim3(grid_for(ni)), dim3(kThreads), 0, s, L.icnt[0], ni);
  hipLaunchKernelGGL(zero_i32, dim3(grid_for(ni)), dim3(kThreads), 0, s, L.icnt[1], ni);
  if (P.np > 0) hipLaunchKernelGGL(cells_build_kernel<T>, dim3(grid_for(P.np)), dim3(kThreads), 0, s, P, L, k);
  return hipGetLastError();
}

// One launch of the step kernel for the run's pusher.
template <int M, typename T, bool D, int WM>
void launch_cells_variant(const StepView& V, const T* E, const T* B, const T* NN, double* dM, double* dE,
                          const RunConsts& k, hipStream_t s) {
  const dim3 grid((unsigned)V.ntiles), block(kThreads);
  if (k.pusher == kPushVay)
    hipLaunchKernelGGL((cells_step_kernel<M, T, D, WM, kPushVay>), grid, block, 0, s, V, E, B, NN, dM, dE, k);
  else if (k.pusher == kPushHC)
    hipLaunchKernelGGL((cells_step_kernel<M, T, D, WM, kPushHC>), grid, block, 0, s, V, E, B, NN, dM, dE, k);
  else
    hipLaunchKernelGGL((cells_step_kernel<M, T, D, WM, kPushBoris>), grid, block, 0, s, V, E, B, NN, dM, dE, k);
}

template <int M, typename T, int WM>
void launch_cells_shape(const StepView& V, const T* E, const T* B, const T* NN, double* dM, double* dE,
                        const RunConsts& k, hipStream_t s) {
  if (dM) launch_cells_variant<M, T, true, WM>(V, E, B, NN, dM, dE, k, s);
  else launch_cells_variant<M, T, false, WM>(V, E, B, NN, dM, dE, k, s);
}

template <int M, typename T>
void launch_cells_mode(int wm, const StepView& V, const T* E, const T* B, const T* NN, double* dM, double* dE,
                       const RunConsts& k, hipStream_t s) {
  if (wm == kLosses) launch_cells_shape<M, T, kLosses>(V, E, B, NN, dM, dE, k, s);
  else if (wm == kWeights) launch_cells_shape<M, T, kWeights>(V, E, B, NN, dM, dE, k, s);
  else launch_cells_shape<M, T, kNoWeights>(V, E, B, NN, dM, dE, k, s);
}

template <typename T>
hipError_t launch_cells_step(int shape, CellLists& L, const T* E, const T* B, const T* NN, bool weights, double* dM,
                             double* dE, const GasLink& gas, const RunConsts& k, hipStream_t s, hipEvent_t before,
                             hipEvent_t after, bool accumulate, bool post) {
  const StepView V = step_view(L, accumulate && dM != nullptr);
  if ((NN || weights) && !(L.buf[0].w && L.buf[1].w)) return hipErrorInvalidValue;
  const int wm = NN ? kLosses : (weights ? kWeights : kNoWeights);
  if (before) (void)hipEventRecord(before, s);
  if (shape == kShapeCIC) launch_cells_mode<2, T>(wm, V, E, B, NN, dM, dE, k, s);
  else launch_cells_mode<3, T>(wm, V, E, B, NN, dM, dE, k, s);
  if (after) (void)hipEventRecord(after, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the exchange of the call's steps goes into the grid once they are done (every step
  // when coupled to the gas); the kernel also clears the consumed overflow counter
  double* pM = post ? dM : nullptr;
  const int64_t work = pM ? (int64_t)k.ncells : L.ntiles;
  hipLaunchKernelGGL(cells_post_kernel, dim3(grid_for(work)), dim3(kThreads), 0, s, V, pM, dE, gas, k);
  L.cur = 1 - L.cur;
  return hipGetLastError();
}

template <typename T>
hipError_t launch_cells_compact(const Packets<T>& P, CellLists& L, const RunConsts& k, hipStream_t s) {
  const int64_t nc = k.ncells;
  const int64_t nscan = nc + L.ntiles * kParts + 1;
  int32_t* counts = L.scan;
  int32_t* offs = counts + nscan;
  int32_t* tmp = offs + nscan + 1;
  hipLaunchKernelGGL(cells_counts_kernel, dim3(grid_for(nscan)), dim3(kThreads), 0, s, L, nc, counts);
  hipError_t e = launch_exclusive_scan(counts, offs, nscan, tmp, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(scan_total_kernel, dim3(1), dim3(1), 0, s, offs, counts, nscan);
  if (L.ntiles > 0) {
    hipLaunchKernelGGL(cells_compact_buckets_kernel<T>, dim3((unsigned)(L.ntiles * kCellTile)), dim3(kCompactThreads),
                       0, s, P, L, offs, k);
    hipLaunchKernelGGL(cells_compact_parts_kernel<T>, dim3((unsigned)L.ntiles), dim3(kThreads), 0, s, P, L, offs, k);
  }
  hipLaunchKernelGGL(cells_compact_overflow_kernel<T>, dim3(grid_for(L.ocap < 262144 ? L.ocap : 262144)),
                     dim3(kThreads), 0, s, P, L, offs, k);
  return hipGetLastError();
}

#define RSOL_CELLS_INSTANTIATE(T)                                                                                  \
  template hipError_t launch_cells_build<T>(const Packets<T>&, CellLists&, const RunConsts&, hipStream_t);         \
  template hipError_t launch_cells_step<T>(int, CellLists&, const T*, const T*, const T*, bool, double*, double*,  \
                                           const GasLink&, const RunConsts&, hipStream_t, hipEvent_t, hipEvent_t,  \
                                           bool, bool);                                                            \
  template hipError_t launch_cells_compact<T>(const Packets<T>&, CellLists&, const RunConsts&, hipStream_t);

RSOL_CELLS_INSTANTIATE(double)
RSOL_CELLS_INSTANTIATE(float)

}  // namespace rsol
