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
// scatter.  A packet's rank inside its cell comes from the scatter's per-bin
// counter; ranks >= kRankCap go to an overflow area at the tile's end.  Packets
// already in order hit the same bin in neighbouring lanes, so every atomic on a
// bin counter is aggregated over the run of equal keys inside the wavefront.
#include "rsol_sort.hpp"

namespace rsol {

namespace {

constexpr int kBlock = 256;
constexpr int kRankCap = 128;
constexpr int kMaskWords = 8;  // cells_per_tile <= 256
constexpr int kScanThreads = 1024;
constexpr int kScanItems = 4;
constexpr int kScanChunk = kScanThreads * kScanItems;

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

// Bin of every packet, the bin histogram, and each packet's rank inside its bin (the
// counter value its atomic returned).  Packets are read in the previous layout's order,
// so packets that stayed in their cell tend to keep their rank and, with it, their
// position: the scatter then writes mostly contiguous runs.
template <typename T>
__global__ void __launch_bounds__(kBlock) keys_hist_kernel(Packets<T> P, RunConsts k, Tiling t,
                                                           int32_t* __restrict__ keys, int32_t* __restrict__ ranks,
                                                           int32_t* hist) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < P.np; base += stride) {
    const int64_t i = base + threadIdx.x;
    int key = -1;
    if (i < P.np) {
      int home[3];
      home_cell(P, i, k, home);
      key = tile_key(home, t);
      keys[i] = key;
    }
    const int r = aggregated_slot(hist, key);
    if (i < P.np) ranks[i] = r;
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

template <typename T>
__global__ void __launch_bounds__(kBlock) scatter_kernel(Packets<T> src, Packets<T> dst, Tiling t,
                                                         const int32_t* __restrict__ keys,
                                                         const int32_t* __restrict__ ranks,
                                                         const int32_t* __restrict__ offsets,
                                                         const int32_t* __restrict__ tables, int32_t* ovf,
                                                         int32_t* __restrict__ pos_out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t np = src.np;
  const int cpt = t.cells_per_tile;
  const int tw = table_words(t);
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < np; base += stride) {
    const int64_t i = base + threadIdx.x;
    if (i < np) {
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
      if (dst.u) {  // NULL: only the permutation (ids) is wanted
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
      if (pos_out) pos_out[i] = (int32_t)j;
    }
  }
}

__global__ void zero_i32_kernel(int32_t* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// Exclusive scan of a kScanChunk slice per block; block totals to sums[blockIdx.x].
__global__ void __launch_bounds__(kScanThreads) scan_chunk_kernel(const int32_t* __restrict__ in,
                                                                  int32_t* __restrict__ out, int64_t n,
                                                                  int32_t* __restrict__ sums) {
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
    if (base + j < n) out[base + j] = excl;
    excl += v[j];
  }
}

__global__ void add_block_offsets_kernel(int32_t* __restrict__ out, int64_t n, const int32_t* __restrict__ sums) {
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  const int32_t add = sums[blockIdx.x];
  for (int j = threadIdx.x; j < kScanChunk; j += blockDim.x)
    if (base + j < n) out[base + j] += add;
}

// offsets[n] = total packet count
__global__ void set_last_kernel(int32_t* offsets, int64_t n, int32_t total) { offsets[n] = total; }

inline int grid_for(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

}  // namespace

size_t sort_scratch_ints(const Tiling& t, int64_t np) {
  const int64_t nbins = t.nbins();
  const int64_t nblk = (nbins + kScanChunk - 1) / kScanChunk;
  const int64_t tw = 1 + (t.cells_per_tile + 31) / 32;
  // offsets (nbins+1), block sums (nblk+16), keys (np), ranks (np), overflow (ntiles),
  // rank tables (ntiles * (kRankCap+1) * tw)
  return (size_t)(nbins + 1) + (size_t)(nblk + 16) + 2 * (size_t)np + (size_t)t.ntiles() +
         (size_t)t.ntiles() * (kRankCap + 1) * tw;
}

int64_t max_sort_bins() { return (int64_t)kScanChunk * kScanChunk; }
int max_cells_per_tile() { return 32 * kMaskWords; }

template <typename T>
hipError_t launch_sort(const Packets<T>& src, const Packets<T>& dst, const RunConsts& k, const Tiling& t,
                       int32_t* ints, hipStream_t s, int32_t* pos_out) {
  const int64_t nbins = t.nbins();
  const int64_t nblk = (nbins + kScanChunk - 1) / kScanChunk;
  int32_t* offsets = ints;                 // nbins + 1
  int32_t* sums = offsets + nbins + 1;     // nblk (+16 slack)
  int32_t* keys = sums + nblk + 16;        // np
  int32_t* ranks = keys + src.np;          // np
  int32_t* ovf = ranks + src.np;           // ntiles
  int32_t* tables = ovf + t.ntiles();      // ntiles * (kRankCap+1) * tw
  hipLaunchKernelGGL(zero_i32_kernel, dim3(grid_for(nbins + 1)), dim3(kBlock), 0, s, offsets, nbins + 1);
  hipLaunchKernelGGL(keys_hist_kernel<T>, dim3(grid_for(src.np)), dim3(kBlock), 0, s, src, k, t, keys, ranks,
                     offsets);
  // exclusive scan of the histogram in place
  hipLaunchKernelGGL(scan_chunk_kernel, dim3((unsigned)nblk), dim3(kScanThreads), 0, s, offsets, offsets, nbins,
                     sums);
  if (nblk > 1) {
    hipLaunchKernelGGL(scan_chunk_kernel, dim3(1), dim3(kScanThreads), 0, s, sums, sums, nblk, (int32_t*)nullptr);
    hipLaunchKernelGGL(add_block_offsets_kernel, dim3((unsigned)nblk), dim3(256), 0, s, offsets, nbins, sums);
  }
  hipLaunchKernelGGL(set_last_kernel, dim3(1), dim3(1), 0, s, offsets, nbins, (int32_t)src.np);
  hipLaunchKernelGGL(tile_tables_kernel, dim3((unsigned)t.ntiles()), dim3(256), 0, s, offsets, t, tables, ovf);
  hipLaunchKernelGGL(scatter_kernel<T>, dim3(grid_for(src.np)), dim3(kBlock), 0, s, src, dst, t, keys, ranks,
                     offsets, tables, ovf, pos_out);
  return hipGetLastError();
}

size_t exclusive_scan_tmp_ints(int64_t n) { return (size_t)((n + kScanChunk - 1) / kScanChunk) + 16; }

hipError_t launch_exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t nblk = (n + kScanChunk - 1) / kScanChunk;
  if (nblk > kScanChunk) return hipErrorInvalidValue;
  hipLaunchKernelGGL(scan_chunk_kernel, dim3((unsigned)nblk), dim3(kScanThreads), 0, s, in, out, n, tmp);
  if (nblk > 1) {
    hipLaunchKernelGGL(scan_chunk_kernel, dim3(1), dim3(kScanThreads), 0, s, tmp, tmp, nblk, (int32_t*)nullptr);
    hipLaunchKernelGGL(add_block_offsets_kernel, dim3((unsigned)nblk), dim3(256), 0, s, out, n, tmp);
  }
  return hipGetLastError();
}

template hipError_t launch_sort<double>(const Packets<double>&, const Packets<double>&, const RunConsts&,
                                        const Tiling&, int32_t*, hipStream_t, int32_t*);
template hipError_t launch_sort<float>(const Packets<float>&, const Packets<float>&, const RunConsts&,
                                       const Tiling&, int32_t*, hipStream_t, int32_t*);

}  // namespace rsol
