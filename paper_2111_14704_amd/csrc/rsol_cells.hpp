// Cell-list step: packets live in per-cell buckets (ping-pong buffers) and are
// moved to their new cell's bucket by the step itself, so every packet a step
// reads is in the cell it is filed under.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rsol_particles.hpp"

namespace rsol {

constexpr int kCellTile = 4;                         // tile edge (cells)
constexpr int kCellTileCells = 64;                   // cells per tile
constexpr int kRegionEdge = kCellTile + 2;           // tile + one-cell halo
constexpr int kRegionCells = kRegionEdge * kRegionEdge * kRegionEdge;
constexpr int kDirs = 27;                            // 3x3x3 tile offsets, index (dx+1) + 3 (dy+1) + 9 (dz+1)
constexpr int kSelfDir = 13;                         // offset (0, 0, 0)

// One structure-of-arrays packet store: component d of slot j at [d * stride + j].
// FP64 keeps absolute positions x; FP32 keeps the in-cell offset (and, where the
// slot does not imply it, the home cell).
struct SlotArrays {
  double* x;        // FP64 only
  int32_t* cell;    // FP32 inbox/overflow/trash only
  float* off;       // FP32 only
  void* u;          // momentum, precision type
  int32_t* id;
  int64_t stride;   // slots in the store
};

// Sizes and buffers of the cell-list layout (all in the library's scratch).
//
// Every tile has an inbox split by the direction the packets came from: the part
// for direction dir holds packets that moved into the tile from the tile at offset
// -dir... written by exactly one source tile (the one at tile - dir), which takes
// slots from an LDS counter and stores the final count with a plain store.  The
// self part (kSelfDir) takes a tile's own packets whose bucket is full.  Packets
// that find their part full (or moved further than one tile) go to one overflow
// list for the grid.
struct CellLists {
  int ntx, nty, ntz;      // tiles per axis (the last tile along an axis may be partial)
  int64_t ntiles;
  int cap;                // bucket slots per cell
  int per_tile;           // inbox slots per tile (sum of dcap)
  int dcap[kDirs];        // inbox slots per direction
  int doff[kDirs + 1];    // first slot of each direction in a tile's inbox
  int64_t ocap;           // overflow slots (one list for the whole grid)
  SlotArrays bucket[2];   // tile by tile, [slot][cell in tile]: slot s of local cell lc of tile t at (t*cap + s)*64 + lc
  SlotArrays inbox[2];    // slot s of direction d of tile t at t*per_tile + doff[d] + s
  SlotArrays ovf[2];      // overflow list
  SlotArrays trash;       // write target of idle lanes: [8][256] slots
  int32_t* bcnt[2];       // packets per cell
  int32_t* icnt[2];       // packets per (tile, direction) [ntiles*kDirs], then the overflow count
  double* halo;           // [ntiles][4][kRegionCells] per-tile exchange accumulators
  int32_t* scan;          // prefix-sum scratch of the compaction
  int cur;                // buffer holding the current state
};

// Scratch bytes the layout needs.
size_t cell_list_bytes(int nx, int ny, int nz, int64_t np, int precision);
// Carve the layout out of `base` (256-byte aligned, cell_list_bytes long).
CellLists cell_list_carve(int nx, int ny, int nz, int64_t np, int precision, char* base);
// Entries of the compaction's prefix sum (cells, tile directions, overflow).
int64_t cell_list_scan_entries(int nx, int ny, int nz);

// Caller packets -> buffer 0 (counters cleared first).
template <typename T>
hipError_t launch_cells_build(const Packets<T>& P, CellLists& L, const RunConsts& k, hipStream_t s);
// One step: buffer cur -> buffer 1-cur; exchange added into dM/dE if dM != NULL.
// `before`/`after` (may be NULL) are recorded around the step kernel itself.
template <typename T>
hipError_t launch_cells_step(int shape, CellLists& L, const T* E, const T* B, double* dM, double* dE,
                             const RunConsts& k, hipStream_t s, hipEvent_t before, hipEvent_t after);
// Buffer cur -> caller packets, cell-major (buckets by cell, then inboxes, then overflow).
template <typename T>
hipError_t launch_cells_compact(const Packets<T>& P, CellLists& L, const RunConsts& k, hipStream_t s);

}  // namespace rsol
