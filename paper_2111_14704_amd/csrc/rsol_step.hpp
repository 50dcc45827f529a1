// The tiled fused packet step and its launch plan.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rsol_particles.hpp"
#include "rsol_sort.hpp"

namespace rsol {

// How rsol_step runs for one parameter set.
struct StepPlan {
  bool tiled;       // tiled LDS kernel (else one thread per packet with global atomics)
  int tx, ty, tz;   // tile of cells owned by one workgroup
  int halo;         // cells staged around the tile: 1 (stencil) + packet drift between re-sorts
  int block;        // threads per workgroup
  double max_step;  // per-step displacement (cells) beyond which the status word is flagged
};

StepPlan plan_step(int nx, int ny, int nz, int shape, int precision, int sort_every, double courant);

// LDS layout of the staged region: extent rx*ry*rz cells (tile + 2*halo per axis),
// cell (x, y, z) at x + sy*y + sz*z with strides padded against bank conflicts.
struct Region {
  int halo;
  int rx, ry, rz;
  int sy, sz;
  int cells;  // sz * rz: LDS cells allocated per component
};

Region make_region(const StepPlan& plan);

// LDS bytes the tiled kernel needs for this plan.
size_t step_lds_bytes(const StepPlan& plan, int precision);

// One fused step over all tiles.  src: packets as left by the last re-sort (or by the
// previous step); dst: where the updated packets go (same positions).  offsets: the
// bin offsets written by the sort.  dM/dE may be NULL (no exchange deposit).
template <typename T>
hipError_t launch_step_tiled(const StepPlan& plan, int shape, const Tiling& t, const Packets<T>& src,
                             const Packets<T>& dst, const int32_t* offsets, const T* E, const T* B, double* dM,
                             double* dE, const RunConsts& k, hipStream_t s);

}  // namespace rsol
