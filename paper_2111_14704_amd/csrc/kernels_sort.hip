// Cell-binned counting sort of the packets (build-internal; the paper has no
// sort).  Bin = tile-major home cell: the grid is cut into tiles of tx*ty*tz
// cells (numbered x-fastest), cells inside a tile are numbered x-fastest.
// Every tile's packets form one contiguous segment, and inside the segment the
// packets are laid out RANK-MAJOR: first the first packet of every non-empty
// cell (in cell order), then the second packet of every cell holding two or
// more, and so on.  Consecutive packets - the lanes of a wavefront in the step
// kernel - then sit in different cells, so their LDS gathers and LDS deposit
// atomics hit different addresses, while their HBM accesses stay contiguous.
//
// Phases: key + histogram, exclusive scan (bin offsets), per-tile rank tables,
// placement, gather.  A packet's rank inside its cell comes from the histogram's
// per-bin counter; ranks >= kRankCap go to an overflow area at the tile's end.  The
// histogram counts each workgroup's chunk of packets in LDS over the 27 tiles around
// the chunk's first packet (packets sorted by tile before, as between the blocks of
// the differentiation form, stay within it) and adds each occupied bin to the global
// counter once; a packet outside that window takes the global counter directly, with
// one atomic per run of equal keys inside the wavefront.  The placement writes only
// the inverse permutation; the gather then moves the packet state with scattered reads
// and contiguous writes.
#include "rsol_sort.hpp"

namespace rsol {

namespace {

constexpr int kBlock = 256;
constexpr int kRankCap = 128;
constexpr int kMaskWords = 8;  // cells_per_tile <= 256
constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr int kScanChunk = kScanThreads * kScanItems;
constexpr int kHistPer = 8;                     // packets per thread in the histogram
constexpr int kHistChunk = kBlock * kHistPer;   // packets per histogram workgroup
constexpr int kWinTiles = 27;                   // tiles of the histogram's LDS window

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// Offset of this lane inside its run of equal keys, after one atomicAdd per run.
// Inactive lanes pass key < 0 and get -1.
__device__ __forceinline__ int aggregated_slot(int32_t* counters, int key) {
  const int lane = lane_id();
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

__device__ __forceinline__ int tile_key(const int home[3], const Tiling& t) {
  const int tx = home[0] / t.tx, ty = home[1] / t.ty, tz = home[2] / t.tz;
  const int lx = home[0] - tx * t.tx, ly = home[1] - ty * t.ty, lz = home[2] - tz * t.tz;
  const int tile = tx + t.ntx * (ty + t.nty * tz);
  return tile * t.cells_per_tile + lx + t.tx * (ly + t.ty * lz);
}

template <typename T>
__device__ __forceinline__ void home_cell(const Packets<T>& P, int64_t i, const RunConsts& k, int home[3]) {
  if constexpr (is_fp64<T>()) {
    const int n[3] = {k.nx, k.ny, k.nz};
    #pragma unroll
    for (int d = 0; d < 3; ++d) {
      // full modulo: a position outside the box (against the contract) must not address
      // outside the bins
      int hd = (int)floor(P.x[d * P.np + i] * k.inv_dx) % n[d];
      home[d] = hd < 0 ? hd + n[d] : hd;
    }
  } else {
    int c = P.cell[i];
    c = c < 0 ? 0 : (c >= k.ncells ? k.ncells - 1 : c);  // a corrupt index must not address outside the bins
    const int nxy = k.nx * k.ny;
    home[2] = c / nxy;
    const int r = c - home[2] * nxy;
    home[1] = r / k.nx;
    home[0] = r - home[1] * k.nx;
  }
}

// Offset of tile coordinate tc from the window centre c along an axis of n tiles: -1,
// 0 or 1 through the periodic wrap (an axis of one or two tiles uses only 0 and 1, so
// every tile has one offset), or 2 outside the window.
__device__ __forceinline__ int window_offset(int tc, int c, int n) {
  int d = tc - c;
  if (d < 0) d += n;
  if (d <= 1) return d;
  return (n >= 3 && d == n - 1) ? -1 : 2;
}

// Bin of every packet, the bin histogram, and each packet's rank inside its bin.  One
// workgroup per chunk of kHistChunk consecutive packets: those whose tile lies in the
// 27-tile window around the chunk's first packet count in LDS (the LDS atomic's value
// is the packet's rank within the chunk), then each occupied window bin is added to the
// global histogram once and its previous value is the chunk's base there; the others
// take the global counter directly.
template <typename T>
__global__ void __launch_bounds__(kBlock) keys_hist_kernel(Packets<T> P, RunConsts k, Tiling t,
                                                           int32_t* __restrict__ keys, int32_t* __restrict__ ranks,
                                                           int32_t* hist) {
  __shared__ int32_t cnt[kWinTiles * 32 * kMaskWords];  // per window bin: count, then base
  __shared__ int sCentre;
  const int cpt = t.cells_per_tile;
  const int nwin = kWinTiles * cpt;
  const int64_t c0 = (int64_t)blockIdx.x * kHistChunk;
  for (int b = threadIdx.x; b < nwin; b += kBlock) cnt[b] = 0;
  if (threadIdx.x == 0) {
    int centre = 0;
    if (c0 < P.np) {
      int home[3];
      home_cell(P, c0, k, home);
      centre = tile_key(home, t) / cpt;
    }
    sCentre = centre;
  }
  __syncthreads();
  const int ct = sCentre;
  const int cx = ct % t.ntx, cy = (ct / t.ntx) % t.nty, cz = ct / (t.ntx * t.nty);
  int key[kHistPer], bin[kHistPer], loc[kHistPer];
  #pragma unroll
  for (int m = 0; m < kHistPer; ++m) {
    const int64_t i = c0 + (int64_t)m * kBlock + threadIdx.x;
    key[m] = -1;
    bin[m] = -1;
    loc[m] = 0;
    if (i < P.np) {
      int home[3];
      home_cell(P, i, k, home);
      key[m] = tile_key(home, t);
      keys[i] = key[m];
      const int tile = key[m] / cpt, lc = key[m] - tile * cpt;
      const int ox = window_offset(tile % t.ntx, cx, t.ntx);
      const int oy = window_offset((tile / t.ntx) % t.nty, cy, t.nty);
      const int oz = window_offset(tile / (t.ntx * t.nty), cz, t.ntz);
      if (ox < 2 && oy < 2 && oz < 2) {
        bin[m] = ((ox + 1) + 3 * ((oy + 1) + 3 * (oz + 1))) * cpt + lc;
        loc[m] = atomicAdd(&cnt[bin[m]], 1);
      }
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nwin; b += kBlock) {
    const int n = cnt[b];
    if (n > 0) {
      const int w = b / cpt, lc = b - w * cpt;
      const int tx = (cx + w % 3 - 1 + t.ntx) % t.ntx;
      const int ty = (cy + (w / 3) % 3 - 1 + t.nty) % t.nty;
      const int tz = (cz + w / 9 - 1 + t.ntz) % t.ntz;
      cnt[b] = atomicAdd(&hist[(tx + t.ntx * (ty + t.nty * tz)) * cpt + lc], n);
    }
  }
  __syncthreads();
  #pragma unroll
  for (int m = 0; m < kHistPer; ++m) {
    const int64_t i = c0 + (int64_t)m * kBlock + threadIdx.x;
    // every lane of the wave takes part (keys outside the window only, -1 elsewhere)
    const int rf = aggregated_slot(hist, bin[m] < 0 ? key[m] : -1);
    if (i < P.np) ranks[i] = bin[m] >= 0 ? cnt[bin[m]] + loc[m] : rf;
  }
}

__device__ __forceinline__ int table_words(const Tiling& t) { return 1 + (t.cells_per_tile + 31) / 32; }

// Per tile: mask[k] = cells holding more than k packets, M[k] = packets of rank < k.
__global__ void __launch_bounds__(256) tile_tables_kernel(const int32_t* __restrict__ offsets, Tiling t,
                                                          int32_t* __restrict__ tables, int32_t* __restrict__ ovf) {
  __shared__ uint32_t mask[kRankCap][kMaskWords];
  __shared__ int32_t m[kRankCap + 1];
  const int64_t tile = blockIdx.x;
  const int cpt = t.cells_per_tile;
  const int W = table_words(t) - 1;
  for (int j = threadIdx.x; j < kRankCap * kMaskWords; j += blockDim.x) (&mask[0][0])[j] = 0u;
  __syncthreads();
  for (int c = threadIdx.x; c < cpt; c += blockDim.x) {
    const int64_t b = tile * cpt + c;
    int n = offsets[b + 1] - offsets[b];
    if (n > kRankCap) n = kRankCap;
    for (int k = 0; k < n; ++k) atomicOr(&mask[k][c >> 5], 1u << (c & 31));
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kRankCap; k += blockDim.x) {
    int cnt = 0;
    for (int w = 0; w < W; ++w) cnt += __popc(mask[k][w]);
    m[k] = cnt;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int k = 0; k < kRankCap; ++k) {
      const int v = m[k];
      m[k] = run;
      run += v;
    }
    m[kRankCap] = run;
    ovf[tile] = 0;
  }
  __syncthreads();
  const int tw = W + 1;
  int32_t* out = tables + tile * (int64_t)(kRankCap + 1) * tw;
  for (int j = threadIdx.x; j < (kRankCap + 1) * tw; j += blockDim.x) {
    const int k = j / tw, w = j - k * tw;
    out[j] = (w == 0) ? m[k] : (k < kRankCap ? (int32_t)mask[k][w - 1] : 0);
  }
}

// Position in the sorted order of every packet, from its bin, its rank and the tile's
// rank tables: inv[j] = i (and pos_out[i] = j).
__global__ void __launch_bounds__(kBlock) place_kernel(int64_t np, Tiling t, const int32_t* __restrict__ keys,
                                                       const int32_t* __restrict__ ranks,
                                                       const int32_t* __restrict__ offsets,
                                                       const int32_t* __restrict__ tables, int32_t* ovf,
                                                       int32_t* __restrict__ inv, int32_t* __restrict__ pos_out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int cpt = t.cells_per_tile;
  const int tw = table_words(t);
  for (int64_t i = xcd_chunk() * blockDim.x + threadIdx.x; i < np; i += stride) {
    const int key = keys[i];
    const int rank = ranks[i];
    const int tile = key / cpt;
    const int c = key - tile * cpt;
    const int32_t* e = tables + ((int64_t)tile * (kRankCap + 1)) * tw;
    int64_t j = offsets[(int64_t)tile * cpt];
    if (rank < kRankCap) {
      e += (int64_t)rank * tw;
      int before = e[0];
      const int wc = c >> 5;
      for (int w = 0; w < wc; ++w) before += __popc((uint32_t)e[1 + w]);
      before += __popc((uint32_t)e[1 + wc] & ((1u << (c & 31)) - 1u));
      j += before;
    } else {
      j += e[(int64_t)kRankCap * tw] + atomicAdd(&ovf[tile], 1);
    }
    inv[j] = (int32_t)i;
    if (pos_out) pos_out[i] = (int32_t)j;
  }
}

// dst[j] = src[inv[j]]: scattered reads, contiguous writes (dst.u NULL: the ids only;
// order_out, optional: a second copy of the ids).
template <typename T>
__global__ void __launch_bounds__(kBlock) gather_kernel(Packets<T> src, Packets<T> dst,
                                                        const int32_t* __restrict__ inv,
                                                        int32_t* __restrict__ order_out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t np = src.np;
  for (int64_t j = xcd_chunk() * blockDim.x + threadIdx.x; j < np; j += stride) {
    const int64_t i = inv[j];
    if (i < 0 || i >= np) continue;  // not a placed position (only a corrupt sort leaves one)
    if (dst.u) {
      if constexpr (is_fp64<T>()) {
        #pragma unroll
        for (int d = 0; d < 3; ++d) dst.x[d * np + j] = src.x[d * np + i];
      } else {
        dst.cell[j] = src.cell[i];
        #pragma unroll
        for (int d = 0; d < 3; ++d) dst.off[d * np + j] = src.off[d * np + i];
      }
      #pragma unroll
      for (int d = 0; d < 3; ++d) dst.u[d * np + j] = src.u[d * np + i];
    }
    dst.id[j] = src.id[i];
    if (order_out) order_out[j] = src.id[i];
  }
}

__global__ void zero_i32_kernel(int32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// Exclusive scan of a kScanChunk slice per block; block totals to sums[blockIdx.x]; copy
// (optional) takes the same values, final when there is one block.
__global__ void __launch_bounds__(kScanThreads) scan_chunk_kernel(const int32_t* __restrict__ in,
                                                                  int32_t* __restrict__ out, int64_t n,
                                                                  int32_t* __restrict__ sums,
                                                                  int32_t* __restrict__ copy) {
  __shared__ int32_t wave_tot[kScanThreads / 64];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
  int32_t v[kScanItems];
  int32_t local = 0;
  #pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    v[j] = (base + j < n) ? in[base + j] : 0;
    local += v[j];
  }
  // inclusive scan of 'local' across the wavefront
  const int lane = lane_id();
  int32_t incl = local;
  #pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int32_t y = __shfl_up(incl, off);
    if (lane >= off) incl += y;
  }
  const int wave = threadIdx.x / 64;
  if (lane == 63) wave_tot[wave] = incl;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t run = 0;
    for (int w = 0; w < kScanThreads / 64; ++w) {
      const int32_t t = wave_tot[w];
      wave_tot[w] = run;
      run += t;
    }
    if (sums) sums[blockIdx.x] = run;
  }
  __syncthreads();
  int32_t excl = wave_tot[wave] + incl - local;
  #pragma unroll
  for (int j = 0; j < kScanItems; ++j) {
    if (base + j < n) {
      out[base + j] = excl;
      if (copy) copy[base + j] = excl;
    }
    excl += v[j];
  }
}

__global__ void add_block_offsets_kernel(int32_t* __restrict__ out, int64_t n, const int32_t* __restrict__ sums,
                                         int32_t* __restrict__ copy) {
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  const int32_t add = sums[blockIdx.x];
  for (int j = threadIdx.x; j < kScanChunk; j += blockDim.x)
    if (base + j < n) {
      const int32_t v = out[base + j] + add;
      out[base + j] = v;
      if (copy) copy[base + j] = v;
    }
}

// offsets[n] = total packet count (and in copy, optional)
__global__ void set_last_kernel(int32_t* offsets, int64_t n, int32_t total, int32_t* copy) {
  offsets[n] = total;
  if (copy) copy[n] = total;
}

inline int grid_for(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

}  // namespace

size_t sort_scratch_ints(const Tiling& t, int64_t np) {
  const int64_t nbins = t.nbins();
  const int64_t nblk = (nbins + kScanChunk - 1) / kScanChunk;
  const int64_t tw = 1 + (t.cells_per_tile + 31) / 32;
  // offsets (nbins+1), block sums (nblk+16), keys (np), ranks (np), inverse
  // permutation (np), overflow (ntiles), rank tables (ntiles * (kRankCap+1) * tw)
  return (size_t)(nbins + 1) + (size_t)(nblk + 16) + 3 * (size_t)np + (size_t)t.ntiles() +
         (size_t)t.ntiles() * (kRankCap + 1) * tw;
}

int64_t max_sort_bins() { return (int64_t)kScanChunk * kScanChunk; }
int max_cells_per_tile() { return 32 * kMaskWords; }

template <typename T>
hipError_t launch_sort(const Packets<T>& src, const Packets<T>& dst, const RunConsts& k, const Tiling& t,
                       int32_t* ints, hipStream_t s, int32_t* pos_out, int32_t* order_out, int32_t* offsets_out) {
  const int64_t nbins = t.nbins();
  const int64_t nblk = (nbins + kScanChunk - 1) / kScanChunk;
  int32_t* offsets = ints;                 // nbins + 1
  int32_t* sums = offsets + nbins + 1;     // nblk (+16 slack)
  int32_t* keys = sums + nblk + 16;        // np
  int32_t* ranks = keys + src.np;          // np
  int32_t* inv = ranks + src.np;           // np
  int32_t* ovf = inv + src.np;             // ntiles
  int32_t* tables = ovf + t.ntiles();      // ntiles * (kRankCap+1) * tw
  hipLaunchKernelGGL(zero_i32_kernel, dim3(grid_for(nbins + 1)), dim3(kBlock), 0, s, offsets, nbins + 1);
  const int64_t hblocks = (src.np + kHistChunk - 1) / kHistChunk;
  hipLaunchKernelGGL(keys_hist_kernel<T>, dim3((unsigned)(hblocks < 1 ? 1 : hblocks)), dim3(kBlock), 0, s, src, k,
                     t, keys, ranks, offsets);
  // exclusive scan of the histogram in place, offsets[nbins] = np
  hipLaunchKernelGGL(scan_chunk_kernel, dim3((unsigned)nblk), dim3(kScanThreads), 0, s, offsets, offsets, nbins,
                     sums, nblk > 1 ? (int32_t*)nullptr : offsets_out);
  if (nblk > 1) {
    hipLaunchKernelGGL(scan_chunk_kernel, dim3(1), dim3(kScanThreads), 0, s, sums, sums, nblk, (int32_t*)nullptr,
                       (int32_t*)nullptr);
    hipLaunchKernelGGL(add_block_offsets_kernel, dim3((unsigned)nblk), dim3(256), 0, s, offsets, nbins, sums,
                       offsets_out);
  }
  hipLaunchKernelGGL(set_last_kernel, dim3(1), dim3(1), 0, s, offsets, nbins, (int32_t)src.np, offsets_out);
  hipLaunchKernelGGL(tile_tables_kernel, dim3((unsigned)t.ntiles()), dim3(256), 0, s, offsets, t, tables, ovf);
  hipLaunchKernelGGL(place_kernel, dim3(grid_for(src.np)), dim3(kBlock), 0, s, src.np, t, keys, ranks, offsets,
                     tables, ovf, inv, pos_out);
  hipLaunchKernelGGL(gather_kernel<T>, dim3(grid_for(src.np)), dim3(kBlock), 0, s, src, dst, inv, order_out);
  return hipGetLastError();
}

size_t exclusive_scan_tmp_ints(int64_t n) { return (size_t)((n + kScanChunk - 1) / kScanChunk) + 16; }

hipError_t launch_exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nblk = (n + kScanChunk - 1) / kScanChunk;
  if (nblk > kScanChunk) return hipErrorInvalidValue;
  hipLaunchKernelGGL(scan_chunk_kernel, dim3((unsigned)nblk), dim3(kScanThreads), 0, s, in, out, n, tmp,
                     (int32_t*)nullptr);
  if (nblk > 1) {
    hipLaunchKernelGGL(scan_chunk_kernel, dim3(1), dim3(kScanThreads), 0, s, tmp, tmp, nblk, (int32_t*)nullptr,
                       (int32_t*)nullptr);
    hipLaunchKernelGGL(add_block_offsets_kernel, dim3((unsigned)nblk), dim3(256), 0, s, out, n, tmp,
                       (int32_t*)nullptr);
  }
  return hipGetLastError();
}

template hipError_t launch_sort<double>(const Packets<double>&, const Packets<double>&, const RunConsts&,
                                        const Tiling&, int32_t*, hipStream_t, int32_t*, int32_t*, int32_t*);
template hipError_t launch_sort<float>(const Packets<float>&, const Packets<float>&, const RunConsts&,
                                       const Tiling&, int32_t*, hipStream_t, int32_t*, int32_t*, int32_t*);

}  // namespace rsol
