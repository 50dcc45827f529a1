// Cell-list step: packets live in per-cell buckets (ping-pong buffers) and are
// moved to their new cell's bucket by the step itself, so every packet a step
// reads is in the cell it is filed under.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rsol_launch.hpp"
#include "rsol_particles.hpp"

namespace rsol {

constexpr int kCellTile = 4;                         // tile edge (cells)
constexpr int kCellTileCells = 64;                   // cells per tile
constexpr int kSlotGroup = 4;                        // consecutive bucket slots of a cell in memory
constexpr int kRegionEdge = kCellTile + 2;           // tile + one-cell halo
constexpr int kRegionCells = kRegionEdge * kRegionEdge * kRegionEdge;
constexpr int kDirs = 27;                            // 3x3x3 tile offsets, index (dx+1) + 3 (dy+1) + 9 (dz+1)
constexpr int kSelfDir = 13;                         // offset (0, 0, 0)

// One structure-of-arrays packet store: component d of slot j at [d * stride + j].
// FP64 keeps absolute positions x; FP32 keeps the in-cell offset and the home cell
// (read only where the slot does not imply it).
struct SlotArrays {
  double* x;        // FP64 only
  int32_t* cell;    // FP32 only
  float* off;       // FP32 only
  void* u;          // momentum, precision type
  int32_t* id;
  int64_t stride;   // slots in the store
  void* w;          // packet weights, precision type (NULL when the layout carries none)
};

// Sizes and buffers of the cell-list layout (all in the library's scratch).
//
// Each of the two buffers is ONE slot store (a SlotArrays whose stride is the total
// slot count), cut into ranges: the buckets first, then the tile inboxes, the
// overflow list and a few trash slots that idle lanes write to.  A packet's place
// is therefore a single slot index.
//
// Buckets are laid out tile by tile as [slot group][cell in tile][slot in group]:
// slot s of local cell lc of tile t is ((t*cap/4 + s/4)*64 + lc)*4 + s%4 (cap a
// multiple of 4), so a quad round reads whole cache lines and the packets a cell
// files in one round share a 32-byte sector.  Every tile has an inbox split into 27 parts by the tile
// offset a packet moved by: part dir of tile t holds packets that came from the tile
// at t - dir, which is that part's only writer (slots from an LDS counter, the final
// count stored with a plain store).  The self part (kSelfDir) takes a tile's own
// packets whose bucket is full.  Packets that find their part full, or that moved
// further than one tile, go to the overflow list, which holds every packet.
struct CellLists {
  int ntx, nty, ntz;      // tiles per axis (the last tile along an axis may be partial)
  int64_t ntiles;
  int cap;                // bucket slots per cell
  int per_tile;           // inbox slots per tile (sum of dcap)
  int dcap[kDirs];        // inbox slots per direction
  int doff[kDirs + 1];    // first slot of each direction in a tile's inbox
  int64_t ocap;           // overflow slots
  int64_t ib0, ov0, tr0;  // first slot of the inboxes, the overflow list, the trash
  SlotArrays buf[2];      // the two slot stores (FP32: with a cell array over all slots)
  int32_t* bcnt[2];       // packets per cell
  int32_t* icnt[2];       // packets per (tile, direction) [ntiles*kDirs], then the overflow count
  double* halo;           // [ntiles][4][kRegionCells] per-tile exchange accumulators
  int32_t* scan;          // prefix-sum scratch of the compaction
  int cur;                // buffer holding the current state
};

// Scratch bytes the layout needs (`weights`: the slot stores carry packet weights).
size_t cell_list_bytes(int nx, int ny, int nz, int64_t np, int precision, bool weights);
// Carve the layout out of `base` (256-byte aligned, cell_list_bytes long).
CellLists cell_list_carve(int nx, int ny, int nz, int64_t np, int precision, bool weights, char* base);
// Entries of the compaction's prefix sum (cells, tile directions, overflow).
int64_t cell_list_scan_entries(int nx, int ny, int nz);

// Caller packets -> buffer 0 (counters cleared first); P.w is copied when both P and
// the layout carry weights.
template <typename T>
hipError_t launch_cells_build(const Packets<T>& P, CellLists& L, const RunConsts& k, hipStream_t s);
// One step: buffer cur -> buffer 1-cur; exchange added into dM/dE if dM != NULL.
// With gas.rho set (then dM = gas.mom, dE = gas.egas) the kernel that adds the
// exchange into the grid also refreshes the gas field E.  NN (nucleon density per
// cell, precision type) selects the step with catastrophic losses (the layout must
// carry weights).  `before`/`after` (may be NULL) are recorded around the step kernel.
template <typename T>
hipError_t launch_cells_step(int shape, CellLists& L, const T* E, const T* B, const T* NN, double* dM, double* dE,
                             const GasLink& gas, const RunConsts& k, hipStream_t s, hipEvent_t before,
                             hipEvent_t after);
// Buffer cur -> caller packets, cell-major (buckets by cell, then inboxes, then overflow).
template <typename T>
hipError_t launch_cells_compact(const Packets<T>& P, CellLists& L, const RunConsts& k, hipStream_t s);

}  // namespace rsol
