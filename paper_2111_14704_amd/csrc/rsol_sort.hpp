// Cell-binned counting sort and the tiling it orders packets by.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rsol_particles.hpp"

namespace rsol {

// Tiles of tx*ty*tz cells covering the grid (the last tile along an axis may be
// partial); ntx*nty*ntz tiles.  Bin of a packet = tile * cells_per_tile + cell in tile.
struct Tiling {
  int tx, ty, tz;
  int ntx, nty, ntz;
  int cells_per_tile;
  __host__ __device__ int64_t ntiles() const { return (int64_t)ntx * nty * ntz; }
  __host__ __device__ int64_t nbins() const { return ntiles() * cells_per_tile; }
};

inline Tiling make_tiling(int nx, int ny, int nz, int tx, int ty, int tz) {
  Tiling t;
  t.tx = tx < nx ? tx : nx;
  t.ty = ty < ny ? ty : ny;
  t.tz = tz < nz ? tz : nz;
  t.ntx = (nx + t.tx - 1) / t.tx;
  t.nty = (ny + t.ty - 1) / t.ty;
  t.ntz = (nz + t.tz - 1) / t.tz;
  t.cells_per_tile = t.tx * t.ty * t.tz;
  return t;
}

// int32 words of scratch the sort needs for this tiling and np packets.
size_t sort_scratch_ints(const Tiling& t, int64_t np);
// Largest bin count the two-level scan handles, and the largest tile the rank tables cover.
int64_t max_sort_bins();
int max_cells_per_tile();

// Exclusive prefix sum of n int32 values (in == out allowed); tmp holds
// exclusive_scan_tmp_ints(n) words.  n is at most max_sort_bins().
size_t exclusive_scan_tmp_ints(int64_t n);
hipError_t launch_exclusive_scan(const int32_t* in, int32_t* out, int64_t n, int32_t* tmp, hipStream_t s);

// Sort src into dst by tile, rank-major inside each tile (dst.u NULL: only dst.id, the
// permutation, is written).  ints = scratch of
// sort_scratch_ints words; on return ints[0..nbins] holds the exclusive bin offsets
// (ints[nbins] = np), so tile t occupies [ints[t*cells_per_tile], ints[(t+1)*cells_per_tile]).
// pos_out (optional, np words): the position in dst of each src packet; order_out
// (optional, np words): a copy of dst.id; offsets_out (optional, nbins + 1 words): a
// copy of the bin offsets.
template <typename T>
hipError_t launch_sort(const Packets<T>& src, const Packets<T>& dst, const RunConsts& k, const Tiling& t,
                       int32_t* ints, hipStream_t s, int32_t* pos_out = nullptr, int32_t* order_out = nullptr,
                       int32_t* offsets_out = nullptr);

}  // namespace rsol
