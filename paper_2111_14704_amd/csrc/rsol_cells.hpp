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
constexpr int kParts = kDirs + 1;                    // inbox parts of a tile: one per offset, then the return part
constexpr int kReturnPart = kDirs;                   // filled with global atomics, from any workgroup

// One packet store: one record per slot, so that a lane moves a packet with a few
// 16-byte loads or stores into one contiguous record and a packet stored alone (a
// mover in an inbox part) fills whole 32-byte sectors:
//   FP64 48 bytes: a = {x, y}, b = {z, u_x}, c = {u_y, u_z} (double pairs), then id (int32)
//     in an array of its own
//   FP32 32 bytes: a = {off_x, off_y, off_z, id bits}, b = {u_x, u_y, u_z, home cell bits}
// (a, b, c point at the record array plus 0, 16, 32 bytes), plus the packet weights
// (precision type) when the layout carries them.  A bucket slot implies its cell; inbox
// and overflow slots keep it (FP32) or imply it by the position (FP64).
struct SlotArrays {
  void* a;
  void* b;
  void* c;        // FP64 only
  int32_t* id;    // FP64 only
  void* w;        // packet weights, precision type (NULL when the layout carries none)
  int64_t stride; // slots in the store
};

// Sizes and buffers of the cell-list layout (all in the library's scratch).
//
// Each of the two buffers is ONE slot store (a SlotArrays whose stride is the total
// slot count), cut into ranges: the buckets first, then the tile inboxes and the
// overflow list.  A packet's place is therefore a single slot index.
//
// Buckets are laid out tile by tile as [slot group][cell in tile][slot in group]:
// slot s of local cell lc of tile t is ((t*cap/4 + s/4)*64 + lc)*4 + s%4 (cap a
// multiple of 4), so a quad round reads whole cache lines.  A bucket holds the packets
// that stayed in their cell during the last step, in the order they were taken.  Every
// tile has an inbox split into 27 parts by the tile offset a packet moved by: part dir
// of tile t holds packets that came from the tile at t - dir, which is that part's only
// writer (slots from an LDS counter, the final count stored with a plain store).  The
// self part (kSelfDir) takes a tile's own packets that changed cell, and those whose
// bucket is full.  Packets that find their part full, or that moved further than one
// tile, and the packets of the overflow list go to the return part of their new tile,
// which any workgroup fills through a global counter; when that is full too, to the
// overflow list.
struct CellLists {
  int ntx, nty, ntz;      // tiles per axis (the last tile along an axis may be partial)
  int64_t ntiles;
  int cap;                // bucket slots per cell
  int per_tile;           // inbox slots per tile (sum of dcap)
  int dcap[kParts];       // inbox slots per part
  int doff[kParts + 1];   // first slot of each part in a tile's inbox
  int64_t ocap;           // overflow slots
  int64_t ib0, ov0, tr0;  // first slot of the inboxes, of the overflow list, and the slot count
  SlotArrays buf[2];      // the two slot stores (FP32: with a cell array over all slots)
  int32_t* bcnt[2];       // packets per cell
  int32_t* icnt[2];       // packets per (tile, part) [ntiles*kParts], then the overflow count
  double* halo;           // [ntiles][4][kRegionCells] per-tile exchange accumulators
  int32_t* scan;          // prefix-sum scratch of the compaction
  int cur;                // buffer holding the current state
};

// Scratch bytes the layout needs (`weights`: the slot stores carry packet weights).
size_t cell_list_bytes(int nx, int ny, int nz, int64_t np, int precision, bool weights);
// Whether the id and weight arrays of the layout's slot stores stay below 4 GiB (the
// step kernel addresses them by 32-bit byte offsets; records by 64-bit ones).
bool cell_list_fits(int nx, int ny, int nz, int64_t np, int precision);
// Carve the layout out of `base` (256-byte aligned, cell_list_bytes long).
CellLists cell_list_carve(int nx, int ny, int nz, int64_t np, int precision, bool weights, char* base);
// Entries of the compaction's prefix sum (cells, tile directions, overflow).
int64_t cell_list_scan_entries(int nx, int ny, int nz);

// Caller packets -> buffer 0 (counters cleared first); P.w is copied when both P and
// the layout carry weights.
template <typename T>
hipError_t launch_cells_build(const Packets<T>& P, CellLists& L, const RunConsts& k, hipStream_t s);
// One step: buffer cur -> buffer 1-cur; exchange deposited if dM != NULL.  The
// step's exchange goes into a per-tile accumulator (added to it when `accumulate`,
// else overwriting it); with `post` a second kernel then adds the accumulators into
// dM/dE, and with gas.rho set (then dM = gas.mom, dE = gas.egas) also refreshes the
// gas field E.  NN (nucleon density per cell, precision type) selects the step with
// catastrophic losses, `weights` the step with per-packet weights (both need a layout
// carrying weights).  `before`/`after` (may be NULL) are recorded around the step
// kernel.
template <typename T>
hipError_t launch_cells_step(int shape, CellLists& L, const T* E, const T* B, const T* NN, bool weights, double* dM,
                             double* dE, const GasLink& gas, const RunConsts& k, hipStream_t s, hipEvent_t before,
                             hipEvent_t after, bool accumulate, bool post);
// Buffer cur -> caller packets, cell-major (buckets by cell, then inboxes, then overflow).
template <typename T>
hipError_t launch_cells_compact(const Packets<T>& P, CellLists& L, const RunConsts& k, hipStream_t s);

}  // namespace rsol
