// C-ABI entry points of librsol: argument validation, scratch carve-up, launch
// sequencing on the caller's stream and status reporting.
#include <math.h>
#include <string.h>

#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/rsol.h"
#include "rsol_adjoint.hpp"
#include "rsol_cells.hpp"
#include "rsol_launch.hpp"
#include "rsol_sort.hpp"
#include "rsol_step.hpp"

using namespace rsol;

struct rsol_ctx {
  rsol_params p;
  int64_t np;
  hipStream_t stream;
  char* scratch;
  size_t scratch_bytes;
  // scratch regions
  uint32_t* status;
  unsigned long long* red;
  int32_t* sort_ints;
  void* perm;           // permuted packet copy written by the sort
  float* E32;
  float* B32;
  char* cells_base;     // cell-list buffers of the default step path
  int32_t* iota;        // 0..np-1: recorded packet indices for the adjoint's sort
  int32_t* spill;       // packets a tiled reverse step leaves to the global kernel (two counts, then indices)
  float* nn32;          // FP32 copy of the nucleon density (FP32 form with RSOL_FLAG_LOSSES)
  // registered caller arrays
  const double* E;
  const double* B;
  void* pos;
  float* off;
  void* u;
  int32_t* id;
  const double* nn;     // catastrophic losses: nucleon density per cell, packet weights, sigma
  void* w;
  double sigma;
  bool have_fields, have_packets, sorted_valid, have_losses;
  bool have_weights;    // per-packet weights registered (rsol_set_weights, or with the losses)
  bool cells_valid;     // the cell lists hold the packets (as of the last rsol_step return)
  bool arrays_stale;    // resident lists hold newer packets than the registered arrays
  int steps_since_sort;
  Tiling tiling;
  StepPlan plan;
  CellLists cells;
  std::string err;
  // optional launch timing: event pairs around every step / sort launch
  bool timing;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev_step, ev_sort;
};

namespace {

thread_local std::string g_init_error;

constexpr size_t kAlign = 256;

size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

int fail(rsol_ctx* h, int code, const std::string& msg) {
  if (h)
    h->err = msg;
  else
    g_init_error = msg;
  return code;
}

int hip_fail(rsol_ctx* h, hipError_t e, const char* where) {
  return fail(h, RSOL_EHIP, std::string(where) + ": " + hipGetErrorString(e));
}

#define RSOL_HIP(h, call, where)               \
  do {                                          \
    hipError_t _e = (call);                     \
    if (_e != hipSuccess) return hip_fail(h, _e, where); \
  } while (0)

int64_t n_cells(const rsol_params& p) { return (int64_t)p.nx * p.ny * p.nz; }

hipEvent_t take_event(rsol_ctx* h) {
  if (!h->ev_pool.empty()) {
    hipEvent_t e = h->ev_pool.back();
    h->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Record the start of a timed launch; returns the pair to close with timed_end.
std::pair<hipEvent_t, hipEvent_t> timed_begin(rsol_ctx* h) {
  std::pair<hipEvent_t, hipEvent_t> pr(nullptr, nullptr);
  if (!h->timing) return pr;
  pr.first = take_event(h);
  pr.second = take_event(h);
  if (pr.first) (void)hipEventRecord(pr.first, h->stream);
  return pr;
}

void timed_end(rsol_ctx* h, std::pair<hipEvent_t, hipEvent_t> pr, bool is_sort) {
  if (!h->timing || !pr.first || !pr.second) return;
  (void)hipEventRecord(pr.second, h->stream);
  (is_sort ? h->ev_sort : h->ev_step).push_back(pr);
}

bool fp32(const rsol_params& p) { return p.precision == RSOL_FP32; }
bool naive(const rsol_params& p) { return (p.flags & RSOL_FLAG_NAIVE) != 0; }
bool loss_layout(const rsol_params& p) { return (p.flags & RSOL_FLAG_LOSSES) != 0; }
constexpr int32_t kKnownFlags = RSOL_FLAG_KEEP_ORDER | RSOL_FLAG_TILED | RSOL_FLAG_NAIVE | RSOL_FLAG_LOSSES |
                                RSOL_FLAG_PUSHER_VAY | RSOL_FLAG_PUSHER_HC | RSOL_FLAG_RESIDENT |
                                RSOL_FLAG_RECORD_ONLY;
int pusher_of(int32_t flags) {
  return (flags & RSOL_FLAG_PUSHER_VAY) ? kPushVay : (flags & RSOL_FLAG_PUSHER_HC) ? kPushHC : kPushBoris;
}
bool tiled_path(int32_t flags) { return (flags & RSOL_FLAG_TILED) && !(flags & RSOL_FLAG_KEEP_ORDER); }
// Flag combinations no path serves; empty when the flags are usable.
std::string flag_conflict(int32_t flags) {
  if ((flags & RSOL_FLAG_PUSHER_VAY) && (flags & RSOL_FLAG_PUSHER_HC)) return "choose one pusher flag";
  if (tiled_path(flags) && pusher_of(flags) != kPushBoris) return "the tiled path runs the Boris pusher only";
  return "";
}

Tiling tiling_for(const rsol_params& p) {
  const StepPlan pl = plan_step(p.nx, p.ny, p.nz, p.shape, p.precision, p.sort_every, p.courant);
  return make_tiling(p.nx, p.ny, p.nz, pl.tx, pl.ty, pl.tz);
}

// Bytes of one sorted packet copy (state and id) for np packets.
size_t packet_copy_bytes(const rsol_params& p, int64_t np) {
  const size_t per = fp32(p) ? (sizeof(int32_t) + 6 * sizeof(float) + sizeof(int32_t))
                             : (6 * sizeof(double) + sizeof(int32_t));
  return per * (size_t)np + 64;
}

// Work buffers of the differentiation form, carved from the cell-list region (which
// holds nothing between rsol_step calls): a second sorted packet copy and two adjoint
// arrays [6][np] (dL/dx rows, then dL/du rows) in tile order.
size_t adj_lam_bytes(const rsol_params& p, int64_t np) {
  return 6 * (size_t)np * (fp32(p) ? sizeof(float) : sizeof(double));
}
size_t adj_work_bytes(const rsol_params& p, int64_t np) {
  return align_up(packet_copy_bytes(p, np)) + 2 * align_up(adj_lam_bytes(p, np));
}

// Scratch layout; returns total bytes and fills offsets when h is given.
size_t layout(const rsol_params& p, int64_t np, rsol_ctx* h) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    size_t at = off;
    off = align_up(off + bytes);
    return at;
  };
  const size_t st = take(sizeof(uint32_t) * 4);
  const size_t rd = take(sizeof(unsigned long long) * 4);
  const Tiling t = tiling_for(p);
  const size_t si = take(sizeof(int32_t) * sort_scratch_ints(t, np));
  const size_t pm = take(packet_copy_bytes(p, np));
  size_t e32 = 0, b32 = 0;
  if (fp32(p)) {
    e32 = take(sizeof(float) * 3 * (size_t)n_cells(p));
    b32 = take(sizeof(float) * 3 * (size_t)n_cells(p));
  }
  const size_t cl_bytes = cell_list_bytes(p.nx, p.ny, p.nz, np, p.precision, loss_layout(p));
  const size_t cl = take(cl_bytes > adj_work_bytes(p, np) ? cl_bytes : adj_work_bytes(p, np));
  const size_t io = take(sizeof(int32_t) * (size_t)np + 64);
  const size_t sp = take(sizeof(int32_t) * (size_t)np + 64);
  const size_t n32 = (fp32(p) && loss_layout(p)) ? take(sizeof(float) * (size_t)n_cells(p)) : 0;
  if (h) {
    char* s = h->scratch;
    h->status = (uint32_t*)(s + st);
    h->red = (unsigned long long*)(s + rd);
    h->sort_ints = (int32_t*)(s + si);
    h->perm = (void*)(s + pm);
    h->E32 = fp32(p) ? (float*)(s + e32) : nullptr;
    h->B32 = fp32(p) ? (float*)(s + b32) : nullptr;
    h->cells_base = s + cl;
    h->iota = (int32_t*)(s + io);
    h->spill = (int32_t*)(s + sp);
    h->nn32 = (fp32(p) && loss_layout(p)) ? (float*)(s + n32) : nullptr;
  }
  return off;
}

std::string validate(const rsol_params* p, int64_t np) {
  if (!p) return "params is NULL";
  if (p->nx < 1 || p->ny < 1 || p->nz < 1 || p->nx > 1024 || p->ny > 1024 || p->nz > 1024)
    return "grid dimensions must be in 1..1024";
  if (p->shape != RSOL_CIC && p->shape != RSOL_TSC) return "shape must be RSOL_CIC or RSOL_TSC";
  if (p->precision != RSOL_FP64 && p->precision != RSOL_FP32) return "precision must be RSOL_FP64 or RSOL_FP32";
  if (p->sort_every < 1 || p->sort_every > 8) return "sort_every must be in 1..8";
  if (p->reserved != 0) return "reserved must be 0";
  if (p->flags & ~kKnownFlags) return "unknown flag bits";
  if (!flag_conflict(p->flags).empty()) return flag_conflict(p->flags);
  if (!(p->dx > 0)) return "dx must be > 0";
  if (!(p->c > 0) || !(p->c_tilde > 0) || p->c_tilde > p->c) return "need 0 < c_tilde <= c";
  if (!isfinite(p->qomc)) return "qomc must be finite";
  if (!(p->dt >= 0) || !isfinite(p->dt)) return "dt must be finite and >= 0";
  if (!(p->courant > 0) || p->courant > 0.5) return "courant must be in (0, 0.5]";
  if (!(p->mass >= 0) || !isfinite(p->mass)) return "mass must be finite and >= 0";
  if (np < 0 || np > (int64_t)INT32_MAX - 64) return "n_particles out of range";
  const Tiling t = tiling_for(*p);
  if (t.nbins() > max_sort_bins()) return "grid too large for the sort";
  if (t.cells_per_tile > max_cells_per_tile()) return "tile larger than the sort supports";
  const int64_t ntiles4 = (int64_t)((p->nx + 3) / 4) * ((p->ny + 3) / 4) * ((p->nz + 3) / 4);
  if (n_cells(*p) + ntiles4 + 1 > max_sort_bins()) return "grid too large for the cell lists";
  if (!cell_list_fits(p->nx, p->ny, p->nz, np, p->precision)) return "too many packets for the cell lists";
  return "";
}

RunConsts consts(const rsol_ctx* h) {
  const rsol_params& p = h->p;
  RunConsts k;
  k.nx = p.nx;
  k.ny = p.ny;
  k.nz = p.nz;
  k.ncells = (int)n_cells(p);
  k.dx = p.dx;
  k.inv_dx = 1.0 / p.dx;
  k.Lx = p.nx * p.dx;
  k.Ly = p.ny * p.dx;
  k.Lz = p.nz * p.dx;
  k.c = p.c;
  k.c_tilde = p.c_tilde;
  k.qomc = p.qomc;
  k.dt = p.dt;
  k.mass = p.mass;
  k.cdt = p.c_tilde * p.dt;
  k.cdt_dx = p.c_tilde * p.dt / p.dx;
  const double vol = p.dx * p.dx * p.dx;
  if (naive(p)) {
    // du/dt = (q/(m c)) [(c/c_tilde) E + beta x B], packet momentum M c_tilde u and
    // energy M c_tilde^2 gamma, no c/c_tilde on the back-reaction
    k.h = 0.5 * (p.c / p.c_tilde) * p.qomc * p.dt;
    k.hb = 0.5 * p.qomc * p.dt;
    k.pc = p.c_tilde;
    k.pfac = -p.mass * p.c_tilde / vol;
    k.efac = -p.mass * p.c_tilde * p.c_tilde / vol;
  } else {
    k.h = 0.5 * (p.c_tilde / p.c) * p.qomc * p.dt;
    k.hb = k.h;
    k.pc = p.c;
    k.pfac = -(p.c / p.c_tilde) * p.mass * p.c / vol;
    k.efac = -(p.c / p.c_tilde) * p.mass * p.c * p.c / vol;
  }
  // a packet may never cross more than one cell per step; the tiled kernel's halo
  // additionally relies on the Courant bound (at most C cells per step)
  k.lrate = h->have_losses ? (p.c_tilde / p.c) * h->sigma * p.c * p.dt : 0.0;
  k.pusher = pusher_of(p.flags);
  k.max_step = h->plan.max_step;
  k.status = h->status;
  return k;
}

template <typename T>
Packets<T> caller_packets(const rsol_ctx* h) {
  Packets<T> P;
  P.np = h->np;
  if constexpr (is_fp64<T>()) {
    P.x = (double*)h->pos;
    P.cell = nullptr;
    P.off = nullptr;
  } else {
    P.x = nullptr;
    P.cell = (int32_t*)h->pos;
    P.off = h->off;
  }
  P.u = (T*)h->u;
  P.id = h->id;
  P.w = h->have_weights ? (T*)h->w : nullptr;
  return P;
}

// A sorted packet copy (the layout packet_copy_bytes sizes) starting at b.
template <typename T>
Packets<T> packets_at(const rsol_ctx* h, char* b) {
  Packets<T> P;
  P.np = h->np;
  const size_t n = (size_t)h->np;
  if constexpr (is_fp64<T>()) {
    P.x = (double*)b;
    P.cell = nullptr;
    P.off = nullptr;
    P.u = (T*)(b + 3 * n * sizeof(double));
    P.id = (int32_t*)(b + 6 * n * sizeof(double));
  } else {
    P.x = nullptr;
    P.cell = (int32_t*)b;
    P.off = (float*)(b + n * sizeof(int32_t));
    P.u = (T*)(b + n * sizeof(int32_t) + 3 * n * sizeof(float));
    P.id = (int32_t*)(b + n * sizeof(int32_t) + 6 * n * sizeof(float));
  }
  return P;
}

template <typename T>
Packets<T> perm_packets(const rsol_ctx* h) { return packets_at<T>(h, (char*)h->perm); }

// The differentiation form's second sorted copy and its adjoint arrays (which = 0, 1).
template <typename T>
Packets<T> adj_packets2(const rsol_ctx* h) { return packets_at<T>(h, h->cells_base); }
template <typename T>
T* adj_lam(const rsol_ctx* h, int which) {
  return (T*)(h->cells_base + align_up(packet_copy_bytes(h->p, h->np)) + which * align_up(adj_lam_bytes(h->p, h->np)));
}

int need(rsol_ctx* h, bool fields, bool packets) {
  if (!h) return fail(nullptr, RSOL_EINVAL, "handle is NULL");
  if (fields && !h->have_fields) return fail(h, RSOL_ESTATE, "fields not registered (rsol_set_fields)");
  if (packets && !h->have_packets) return fail(h, RSOL_ESTATE, "packets not registered (rsol_set_particles)");
  return RSOL_OK;
}

// The tiled path carries no packet weights.
int losses_path_ok(rsol_ctx* h) {
  if (h->have_weights && (h->p.flags & RSOL_FLAG_TILED) && !(h->p.flags & RSOL_FLAG_KEEP_ORDER))
    return fail(h, RSOL_EINVAL, "the tiled path does not carry packet weights or losses");
  return RSOL_OK;
}

template <typename T>
const T* field_E(const rsol_ctx* h) {
  if constexpr (is_fp64<T>()) return h->E; else return h->E32;
}
template <typename T>
const T* field_B(const rsol_ctx* h) {
  if constexpr (is_fp64<T>()) return h->B; else return h->B32;
}
// nucleon density of the loss step, or NULL without losses
template <typename T>
const T* field_NN(const rsol_ctx* h) {
  if (!h->have_losses) return nullptr;
  if constexpr (is_fp64<T>()) return h->nn; else return h->nn32;
}

// Copy the permuted packets back over the caller's arrays.
template <typename T>
int copy_back(rsol_ctx* h) {
  const Packets<T> src = perm_packets<T>(h), dst = caller_packets<T>(h);
  const size_t n = (size_t)h->np;
  if (n == 0) return RSOL_OK;
  if constexpr (is_fp64<T>()) {
    RSOL_HIP(h, hipMemcpyAsync(dst.x, src.x, 3 * n * sizeof(double), hipMemcpyDeviceToDevice, h->stream), "copy x");
  } else {
    RSOL_HIP(h, hipMemcpyAsync(dst.cell, src.cell, n * sizeof(int32_t), hipMemcpyDeviceToDevice, h->stream), "copy cell");
    RSOL_HIP(h, hipMemcpyAsync(dst.off, src.off, 3 * n * sizeof(float), hipMemcpyDeviceToDevice, h->stream), "copy off");
  }
  RSOL_HIP(h, hipMemcpyAsync(dst.u, src.u, 3 * n * sizeof(T), hipMemcpyDeviceToDevice, h->stream), "copy u");
  RSOL_HIP(h, hipMemcpyAsync(dst.id, src.id, n * sizeof(int32_t), hipMemcpyDeviceToDevice, h->stream), "copy id");
  return RSOL_OK;
}

template <typename T>
int do_sort(rsol_ctx* h, bool copy) {
  if (h->np == 0) {
    h->sorted_valid = true;
    h->steps_since_sort = 0;
    return RSOL_OK;
  }
  const RunConsts k = consts(h);
  auto ev = timed_begin(h);
  RSOL_HIP(h, launch_sort<T>(caller_packets<T>(h), perm_packets<T>(h), k, h->tiling, h->sort_ints, h->stream),
           "sort");
  timed_end(h, ev, true);
  h->sorted_valid = true;
  h->steps_since_sort = 0;
  if (copy) return copy_back<T>(h);
  return RSOL_OK;
}

// Default path: caller arrays -> cell buckets, nsteps cell-list steps, buckets ->
// caller arrays (cell-major).
template <typename T>
int do_step_cells(rsol_ctx* h, int32_t nsteps, double* dM, double* dE, const GasLink& gas, bool reuse) {
  const RunConsts k = consts(h);
  const Packets<T> P = caller_packets<T>(h);
  auto ev = timed_begin(h);
  if (!reuse) {
    RSOL_HIP(h, launch_cells_build<T>(P, h->cells, k, h->stream), "cell lists (build)");
    timed_end(h, ev, true);
  }
  for (int32_t s = 0; s < nsteps; ++s) {
    std::pair<hipEvent_t, hipEvent_t> pr(nullptr, nullptr);
    if (h->timing) {
      pr.first = take_event(h);
      pr.second = take_event(h);
    }
    // the per-tile exchange accumulators sum the call's steps and go into dM/dE after
    // the last one; a step coupled to the gas needs its exchange in the gas at once
    const bool accumulate = s > 0 && !gas.rho;
    const bool post = gas.rho || s == nsteps - 1;
    RSOL_HIP(h, launch_cells_step<T>(h->p.shape, h->cells, field_E<T>(h), field_B<T>(h), field_NN<T>(h),
                                     h->have_weights && !h->have_losses, dM, dE, gas, k, h->stream, pr.first,
                                     pr.second, accumulate, post),
             "step (cells)");
    if (pr.first && pr.second) h->ev_step.push_back(pr);
  }
  h->sorted_valid = false;
  if (h->p.flags & RSOL_FLAG_RESIDENT) {
    // the packets stay in the lists; the arrays catch up on the next sync
    h->cells_valid = true;
    h->arrays_stale = true;
    return RSOL_OK;
  }
  ev = timed_begin(h);
  RSOL_HIP(h, launch_cells_compact<T>(P, h->cells, k, h->stream), "cell lists (compact)");
  timed_end(h, ev, true);
  return RSOL_OK;
}

// Copy the packets of resident cell lists back to the registered arrays.
int sync_arrays(rsol_ctx* h) {
  if (!h->arrays_stale) return RSOL_OK;
  const RunConsts k = consts(h);
  auto ev = timed_begin(h);
  if (fp32(h->p))
    RSOL_HIP(h, launch_cells_compact<float>(caller_packets<float>(h), h->cells, k, h->stream), "cell lists (sync)");
  else
    RSOL_HIP(h, launch_cells_compact<double>(caller_packets<double>(h), h->cells, k, h->stream), "cell lists (sync)");
  timed_end(h, ev, true);
  h->arrays_stale = false;
  return RSOL_OK;
}

bool adj_tiled(const rsol_ctx* h);
template <typename T>
int record_tiled(rsol_ctx* h, int32_t nsteps, char* states, const RunConsts& k);

template <typename T>
int do_step(rsol_ctx* h, int32_t nsteps, double* dM, double* dE, const GasLink& gas) {
  const bool reuse = (h->p.flags & RSOL_FLAG_RESIDENT) && h->cells_valid;
  if (!reuse)
    if (int rc = sync_arrays(h)) return rc;
  h->cells_valid = false;
  if ((h->p.flags & (RSOL_FLAG_KEEP_ORDER | RSOL_FLAG_TILED)) == 0)
    return do_step_cells<T>(h, nsteps, dM, dE, gas, reuse);
  const RunConsts k = consts(h);
  // keep-order steps that deposit nothing (the differentiation form's forward pass) run
  // on tile-sorted copies with the fields staged per tile, as its recording does
  if ((h->p.flags & RSOL_FLAG_KEEP_ORDER) && !dM && !dE && !gas.rho && pusher_of(h->p.flags) == kPushBoris &&
      !h->have_losses && h->np > 0 && adj_tiled(h)) {
    h->sorted_valid = false;
    return record_tiled<T>(h, nsteps, nullptr, k);
  }
  const bool global = (h->p.flags & RSOL_FLAG_KEEP_ORDER) != 0 || !h->plan.tiled;
  for (int32_t s = 0; s < nsteps; ++s) {
    if (global) {
      auto ev = timed_begin(h);
      // packet weights without losses: the weighted step with a zero loss rate (its
      // density input is then never used; any grid array of the right size serves)
      const T* nn = h->have_losses ? field_NN<T>(h) : (h->have_weights ? field_B<T>(h) : nullptr);
      RSOL_HIP(h, launch_step_global<T>(h->p.shape, caller_packets<T>(h), field_E<T>(h), field_B<T>(h), nn, dM, dE,
                                        k, h->stream),
               "step (global)");
      timed_end(h, ev, false);
      h->sorted_valid = false;
      if (gas.rho) RSOL_HIP(h, launch_gas_field(gas, n_cells(h->p), h->stream), "gas field");
      continue;
    }
    bool from_perm = false;
    if (!h->sorted_valid || h->steps_since_sort >= h->p.sort_every) {
      int rc = do_sort<T>(h, false);
      if (rc) return rc;
      from_perm = true;
    }
    const Packets<T> src = from_perm ? perm_packets<T>(h) : caller_packets<T>(h);
    auto ev = timed_begin(h);
    RSOL_HIP(h, launch_step_tiled<T>(h->plan, h->p.shape, h->tiling, src, caller_packets<T>(h), h->sort_ints,
                                     field_E<T>(h), field_B<T>(h), dM, dE, k, h->stream),
             "step (tiled)");
    timed_end(h, ev, false);
    h->steps_since_sort += 1;
    if (gas.rho) RSOL_HIP(h, launch_gas_field(gas, n_cells(h->p), h->stream), "gas field");
  }
  return RSOL_OK;
}

// ---------------------------------------------------------------- differentiation form
// Recorded steps come in blocks of kAdjBlock.  At the start of each block the packets are
// counting-sorted by tile (the first block from the caller's arrays, later ones from the
// previous block's sorted copy, which is nearly in order already) and the block's steps
// run on that sorted copy with each tile's fields staged in LDS.  A step's slab holds
// the starting state in its block's order; the first slab of a block also holds the
// block's order (caller index of each position), its bin offsets and, once the next
// block is sorted, the position of each of its packets in the next block's order.  The
// reverse sweep keeps the adjoints in the same orders, so no per-packet access in
// either direction goes through a permutation except at block boundaries.
constexpr int kAdjBlock = 4;
constexpr int kAdjHalo = 2;

struct SlabLayout {
  size_t state, order, next, offsets, total;
};

SlabLayout slab_layout(const rsol_ctx* h) {
  SlabLayout L;
  const size_t n = (size_t)h->np;
  L.state = 0;
  size_t off = align_up(n * (fp32(h->p) ? 7 * sizeof(float) : 6 * sizeof(double)));
  L.order = off;
  off = align_up(off + n * sizeof(int32_t));
  L.next = off;
  off = align_up(off + n * sizeof(int32_t));
  L.offsets = off;
  off = align_up(off + ((size_t)h->tiling.nbins() + 1) * sizeof(int32_t));
  L.total = off;
  return L;
}

bool adj_tiled(const rsol_ctx* h) {
  return step_backward_tiled_fits(h->tiling, kAdjHalo) && step_record_tiled_fits(h->tiling, kAdjHalo);
}

// View of the packet state stored in a slab (ids unused).
template <typename T>
Packets<T> slab_packets(const rsol_ctx* h, const char* at) {
  Packets<T> P;
  P.np = h->np;
  P.id = nullptr;
  if constexpr (is_fp64<T>()) {
    P.x = (double*)at;
    P.cell = nullptr;
    P.off = nullptr;
    P.u = (T*)at + 3 * h->np;
  } else {
    P.x = nullptr;
    P.cell = (int32_t*)at;
    P.off = (float*)at + h->np;
    P.u = (T*)at + 4 * h->np;
  }
  return P;
}


template <typename T>
int record_global(rsol_ctx* h, int32_t nsteps, char* states, const RunConsts& k) {
  const SlabLayout sl = slab_layout(h);
  // RSOL_FLAG_RECORD_ONLY: advance a copy and leave the caller's arrays alone
  Packets<T> P = caller_packets<T>(h);
  if (h->p.flags & RSOL_FLAG_RECORD_ONLY) {
    const Packets<T> c = perm_packets<T>(h);
    const size_t n = (size_t)h->np;
    if constexpr (is_fp64<T>()) {
      RSOL_HIP(h, hipMemcpyAsync(c.x, P.x, 3 * n * sizeof(double), hipMemcpyDeviceToDevice, h->stream), "copy x");
    } else {
      RSOL_HIP(h, hipMemcpyAsync(c.cell, P.cell, n * sizeof(int32_t), hipMemcpyDeviceToDevice, h->stream), "copy cell");
      RSOL_HIP(h, hipMemcpyAsync(c.off, P.off, 3 * n * sizeof(float), hipMemcpyDeviceToDevice, h->stream), "copy off");
    }
    RSOL_HIP(h, hipMemcpyAsync(c.u, P.u, 3 * n * sizeof(T), hipMemcpyDeviceToDevice, h->stream), "copy u");
    P.x = c.x;
    P.cell = c.cell;
    P.off = c.off;
    P.u = c.u;
  }
  for (int32_t n = 0; n < nsteps; ++n)
    RSOL_HIP(h, launch_step_record<T>(h->p.shape, P, field_E<T>(h), field_B<T>(h),
                                      states + (size_t)n * sl.total + sl.state, k, h->stream), "record step");
  return RSOL_OK;
}

// Advance nsteps steps on tile-sorted copies (sorted every kAdjBlock steps) and return
// the packets to the caller's arrays in their order; with states, record every step's
// starting state and each block's ordering there.  When recording, a step reads its
// starting state from its own slab (where the sort or the previous step put it) and
// writes the next state into the next step's slab, or into the scratch copy `cur` at
// the end of a block (the next block's sort reads it) and of the call, so no step copies
// its state separately; without states the steps advance `cur` in place.
template <typename T>
int record_tiled(rsol_ctx* h, int32_t nsteps, char* states, const RunConsts& k) {
  const SlabLayout sl = slab_layout(h);
  Packets<T> cur = perm_packets<T>(h), nxt = adj_packets2<T>(h);
  auto slab_of = [&](int32_t n) { return states + (size_t)n * sl.total; };
  // the state slab of step n as packet arrays carrying the current block's ids
  auto slab_view = [&](int32_t n) {
    Packets<T> P = slab_packets<T>(h, slab_of(n) + sl.state);
    P.id = cur.id;
    return P;
  };
  RSOL_HIP(h, launch_iota(h->iota, h->np, h->stream), "iota");
  for (int32_t n = 0; n < nsteps; ++n) {
    if (n % kAdjBlock == 0) {
      // the sort also writes the block's order and bin offsets into the step's slab
      int32_t* order = states ? (int32_t*)(slab_of(n) + sl.order) : nullptr;
      int32_t* offs = states ? (int32_t*)(slab_of(n) + sl.offsets) : nullptr;
      int32_t* pos = (states && n > 0) ? (int32_t*)(slab_of(n - kAdjBlock) + sl.next) : nullptr;
      Packets<T> src = cur;
      if (n == 0) {
        src = caller_packets<T>(h);
        src.id = h->iota;
        src.w = nullptr;
      }
      Packets<T> dst = nxt;
      if (states) {
        dst = slab_packets<T>(h, slab_of(n) + sl.state);
        dst.id = nxt.id;
      }
      RSOL_HIP(h, launch_sort<T>(src, dst, k, h->tiling, h->sort_ints, h->stream, pos, order, offs), "record sort");
      if (states) {
        // the block's ids now sit in nxt.id; cur keeps its arrays for the block's last step
        int32_t* t = cur.id;
        cur.id = nxt.id;
        nxt.id = t;
      } else {
        const Packets<T> t = cur;
        cur = nxt;
        nxt = t;
      }
    }
    Packets<T> in = cur, out = cur;
    if (states) {
      in = slab_view(n);
      if (n + 1 < nsteps && (n + 1) % kAdjBlock != 0) out = slab_view(n + 1);
    }
    auto ev = timed_begin(h);
    RSOL_HIP(h, launch_step_record_tiled<T>(h->p.shape, in, out, h->sort_ints, h->tiling, kAdjHalo, field_E<T>(h),
                                            field_B<T>(h), k, h->stream),
             "record step");
    timed_end(h, ev, false);
  }
  if (!(states && (h->p.flags & RSOL_FLAG_RECORD_ONLY)))
    RSOL_HIP(h, launch_unsort<T>(cur, caller_packets<T>(h), h->stream), "record unsort");
  return RSOL_OK;
}

template <typename T>
int backward_global(rsol_ctx* h, int32_t nsteps, const char* states, T* lam_x, T* lam_u, const double* lam_dM,
                    const double* lam_dE, double* gE, double* gB, const RunConsts& k) {
  const SlabLayout sl = slab_layout(h);
  for (int32_t n = nsteps - 1; n >= 0; --n) {
    const auto pr = timed_begin(h);
    RSOL_HIP(h, launch_step_backward<T>(h->p.shape, states + (size_t)n * sl.total + sl.state, h->np, lam_x, lam_u,
                                        field_E<T>(h), field_B<T>(h), lam_dM, lam_dE, gE, gB, k, h->stream),
             "step backward");
    timed_end(h, pr, false);
  }
  return RSOL_OK;
}

template <typename T>
int backward_tiled(rsol_ctx* h, int32_t nsteps, const char* states, T* lam_x, T* lam_u, const double* lam_dM,
                   const double* lam_dE, double* gE, double* gB, const RunConsts& k) {
  const SlabLayout sl = slab_layout(h);
  const int64_t np = h->np;
  T* L0 = adj_lam<T>(h, 0);
  T* L1 = adj_lam<T>(h, 1);
  auto first_slab = [&](int b) { return states + (size_t)b * kAdjBlock * sl.total; };
  int block = (nsteps - 1) / kAdjBlock;
  // the caller's adjoints into records in the last block's order
  const int32_t* order = (const int32_t*)(first_slab(block) + sl.order);
  RSOL_HIP(h, launch_records_rows<T>(lam_x, lam_u, L0, L1, order, np, false, h->stream), "adjoint gather");
  RSOL_HIP(h, launch_spill_clear(h->spill, h->stream), "spill clear");
  for (int32_t n = nsteps - 1; n >= 0; --n) {
    const int b = n / kAdjBlock;
    if (b != block) {
      // from block b+1's order into block b's: position j of block b sits at next[j]
      const int32_t* next = (const int32_t*)(first_slab(b) + sl.next);
      RSOL_HIP(h, launch_permute_records<T>(L0, L1, next, np, h->stream), "adjoint reorder");
      T* t = L0;
      L0 = L1;
      L1 = t;
      block = b;
    }
    const int32_t* offsets = (const int32_t*)(first_slab(b) + sl.offsets);
    const Packets<T> slab = slab_packets<T>(h, states + (size_t)n * sl.total + sl.state);
    const int parity = n & 1;
    const auto pr = timed_begin(h);
    RSOL_HIP(h, launch_step_backward_tiled<T>(h->p.shape, slab, offsets, h->tiling, kAdjHalo, h->spill, parity, L0,
                                              field_E<T>(h), field_B<T>(h), lam_dM, lam_dE, gE, gB, k, h->stream),
             "step backward");
    timed_end(h, pr, false);
    RSOL_HIP(h, launch_step_backward_spilled<T>(h->p.shape, slab, h->spill, parity, L0, field_E<T>(h),
                                                field_B<T>(h), lam_dM, lam_dE, gE, gB, k, h->stream),
             "step backward spilled");
  }
  const int32_t* order0 = (const int32_t*)(states + sl.order);
  RSOL_HIP(h, launch_records_rows<T>(lam_x, lam_u, L0, L1, order0, np, true, h->stream), "adjoint scatter");
  return RSOL_OK;
}

// Moments of the caller's packets: sorted by tile (the permutation only) and accumulated
// per tile in LDS, or with global atomics where the tile region does not fit.
template <typename T>
int moments(rsol_ctx* h, double* rho, double* P, double* e) {
  const RunConsts k = consts(h);
  Packets<T> src = caller_packets<T>(h);
  if (!moments_tiled_fits(h->tiling)) {
    RSOL_HIP(h, launch_moments<T>(h->p.shape, src, rho, P, e, k, h->stream), "moments");
    return RSOL_OK;
  }
  Packets<T> ord = perm_packets<T>(h);
  ord.x = nullptr;
  ord.cell = nullptr;
  ord.off = nullptr;
  ord.u = nullptr;
  ord.w = nullptr;
  src.id = h->iota;
  RSOL_HIP(h, launch_iota(h->iota, h->np, h->stream), "iota");
  RSOL_HIP(h, launch_sort<T>(src, ord, k, h->tiling, h->sort_ints, h->stream), "moments sort");
  h->sorted_valid = false;
  RSOL_HIP(h, launch_moments_tiled<T>(h->p.shape, caller_packets<T>(h), ord.id, h->sort_ints, h->tiling, rho, P, e,
                                      k, h->stream), "moments");
  return RSOL_OK;
}

// Fill a new context for np packets over the scratch at `scratch` (bytes long, already
// checked against the layout): carve the regions, the cell lists, clear the status words.
int init_ctx(rsol_ctx* h, const rsol_params* p, int64_t n_particles, void* stream, void* scratch,
             size_t scratch_bytes) {
  h->p = *p;
  h->np = n_particles;
  h->stream = (hipStream_t)stream;
  h->scratch = (char*)scratch;
  h->scratch_bytes = scratch_bytes;
  h->plan = plan_step(p->nx, p->ny, p->nz, p->shape, p->precision, p->sort_every, p->courant);
  h->tiling = make_tiling(p->nx, p->ny, p->nz, h->plan.tx, h->plan.ty, h->plan.tz);
  layout(*p, n_particles, h);
  h->cells = cell_list_carve(p->nx, p->ny, p->nz, n_particles, p->precision, loss_layout(*p), h->cells_base);
  hipError_t e = launch_fill_u32(h->status, 0u, 4, h->stream);
  if (e != hipSuccess) return hip_fail(nullptr, e, "init status");
  return RSOL_OK;
}

// ---------------------------------------------------------------- static scratch
// The scratch of rsol_step_static: a device array of fixed size in the library's code
// object, so that the entry point needs no device allocation.  Host code must not pass
// the array's name to a kernel (on the host it is a stand-in, not a device address):
// static_scratch() looks up its address once per device and every use goes through it.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_static_mu;
char* g_static_ptr[kMaxDevices] = {};

int static_scratch(char** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetDevice");
  if (dev < 0 || dev >= kMaxDevices) return fail(nullptr, RSOL_EINVAL, "device index out of range");
  std::lock_guard<std::mutex> lock(g_static_mu);
  if (!g_static_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(nullptr, e, "hipGetSymbolAddress(scratch)");
    if (!ptr || ((uintptr_t)ptr) % kAlign) return fail(nullptr, RSOL_EHIP, "static scratch address unusable");
    g_static_ptr[dev] = (char*)ptr;
  }
  *out = g_static_ptr[dev];
  return RSOL_OK;
}

}  // namespace

extern "C" {

size_t rsol_scratch_bytes(const rsol_params* p, int64_t n_particles) {
  if (!validate(p, n_particles).empty()) return 0;
  return layout(*p, n_particles, nullptr);
}

int rsol_init(const rsol_params* p, int64_t n_particles, void* stream, void* scratch, size_t scratch_bytes,
              rsol_handle* out) {
  if (!out) return fail(nullptr, RSOL_EINVAL, "out is NULL");
  *out = nullptr;
  const std::string bad = validate(p, n_particles);
  if (!bad.empty()) return fail(nullptr, RSOL_EINVAL, bad);
  const size_t need_bytes = layout(*p, n_particles, nullptr);
  if (!scratch) return fail(nullptr, RSOL_EINVAL, "scratch is NULL");
  if (((uintptr_t)scratch) % kAlign) return fail(nullptr, RSOL_EINVAL, "scratch must be 256-byte aligned");
  if (scratch_bytes < need_bytes)
    return fail(nullptr, RSOL_ESCRATCH,
                "scratch too small: need " + std::to_string(need_bytes) + " bytes, got " + std::to_string(scratch_bytes));
  rsol_ctx* h = new (std::nothrow) rsol_ctx();
  if (!h) return fail(nullptr, RSOL_EINVAL, "out of host memory");
  if (int rc = init_ctx(h, p, n_particles, stream, scratch, scratch_bytes)) {
    delete h;
    return rc;
  }
  *out = h;
  return RSOL_OK;
}

int rsol_step_static(const rsol_params* p, int64_t n_particles, void* stream, const double* E, const double* B,
                     void* pos, float* off, void* u, int32_t* id, int32_t nsteps, double* dM, double* dE) {
  const std::string bad = validate(p, n_particles);
  if (!bad.empty()) return fail(nullptr, RSOL_EINVAL, bad);
  if (!(p->dt > 0)) return fail(nullptr, RSOL_EINVAL, "dt must be > 0 (no Courant timestep is computed here)");
  if (p->flags & (RSOL_FLAG_RESIDENT | RSOL_FLAG_LOSSES))
    return fail(nullptr, RSOL_EINVAL, "RSOL_FLAG_RESIDENT and RSOL_FLAG_LOSSES need a handle");
  if (nsteps < 0) return fail(nullptr, RSOL_EINVAL, "nsteps < 0");
  const size_t need_bytes = layout(*p, n_particles, nullptr);
  if (need_bytes > kStaticScratchBytes)
    return fail(nullptr, RSOL_ESCRATCH,
                "the static scratch holds " + std::to_string(kStaticScratchBytes) + " bytes; this problem needs " +
                    std::to_string(need_bytes));
  char* base = nullptr;
  if (int rc = static_scratch(&base)) return rc;
  rsol_ctx h{};
  if (int rc = init_ctx(&h, p, n_particles, stream, base, kStaticScratchBytes)) return rc;
  int rc = rsol_set_fields(&h, E, B);
  if (!rc) rc = rsol_set_particles(&h, pos, off, u, id);
  if (!rc) rc = rsol_step(&h, nsteps, dM, dE);
  if (rc) g_init_error = h.err;
  return rc;
}

int rsol_destroy(rsol_handle h) {
  if (h) {
    for (auto& pr : h->ev_step) h->ev_pool.push_back(pr.first), h->ev_pool.push_back(pr.second);
    for (auto& pr : h->ev_sort) h->ev_pool.push_back(pr.first), h->ev_pool.push_back(pr.second);
    for (hipEvent_t e : h->ev_pool)
      if (e) (void)hipEventDestroy(e);
  }
  delete h;
  return RSOL_OK;
}

int rsol_timing(rsol_handle h, int32_t enable) {
  if (int rc = need(h, false, false)) return rc;
  h->timing = enable != 0;
  return RSOL_OK;
}

int rsol_timing_read(rsol_handle h, double* step_ms, int64_t* n_step, double* sort_ms, int64_t* n_sort) {
  if (int rc = need(h, false, false)) return rc;
  RSOL_HIP(h, hipStreamSynchronize(h->stream), "timing sync");
  double acc[2] = {0.0, 0.0};
  int64_t cnt[2] = {0, 0};
  for (int which = 0; which < 2; ++which) {
    auto& v = which == 0 ? h->ev_step : h->ev_sort;
    for (auto& pr : v) {
      float ms = 0.f;
      RSOL_HIP(h, hipEventElapsedTime(&ms, pr.first, pr.second), "event elapsed");
      acc[which] += ms;
      cnt[which] += 1;
      h->ev_pool.push_back(pr.first);
      h->ev_pool.push_back(pr.second);
    }
    v.clear();
  }
  if (step_ms) *step_ms = acc[0];
  if (n_step) *n_step = cnt[0];
  if (sort_ms) *sort_ms = acc[1];
  if (n_sort) *n_sort = cnt[1];
  return RSOL_OK;
}

const char* rsol_last_error(rsol_handle h) { return h ? h->err.c_str() : g_init_error.c_str(); }

int rsol_electric_field(rsol_handle h, const double* u_gas, const double* B, double* E) {
  if (int rc = need(h, false, false)) return rc;
  if (!u_gas || !B || !E) return fail(h, RSOL_EINVAL, "NULL field pointer");
  RSOL_HIP(h, launch_electric_field(u_gas, B, E, (int)n_cells(h->p), h->p.c, h->stream), "electric_field");
  return RSOL_OK;
}

int rsol_set_fields(rsol_handle h, const double* E, const double* B) {
  if (int rc = need(h, false, false)) return rc;
  if (!E || !B) return fail(h, RSOL_EINVAL, "NULL field pointer");
  h->E = E;
  h->B = B;
  if (fp32(h->p)) {
    RSOL_HIP(h, launch_to_fp32(E, h->E32, 3 * n_cells(h->p), h->stream), "E to fp32");
    RSOL_HIP(h, launch_to_fp32(B, h->B32, 3 * n_cells(h->p), h->stream), "B to fp32");
  }
  h->have_fields = true;
  return RSOL_OK;
}

int rsol_set_losses(rsol_handle h, double sigma, const double* nn, void* w) {
  if (int rc = need(h, false, false)) return rc;
  if (int rc = sync_arrays(h)) return rc;
  h->cells_valid = false;  // the packets change (or the cell-list scratch is reused)
  if (!loss_layout(h->p)) return fail(h, RSOL_ESTATE, "handle created without RSOL_FLAG_LOSSES");
  if (!(sigma >= 0) || !isfinite(sigma)) return fail(h, RSOL_EINVAL, "sigma must be finite and >= 0");
  if (!nn || (!w && h->np > 0)) return fail(h, RSOL_EINVAL, "NULL loss array");
  if (h->p.flags & RSOL_FLAG_TILED && !(h->p.flags & RSOL_FLAG_KEEP_ORDER))
    return fail(h, RSOL_EINVAL, "the tiled path does not carry losses");
  h->sigma = sigma;
  h->nn = nn;
  h->w = w;
  if (fp32(h->p)) RSOL_HIP(h, launch_to_fp32(nn, h->nn32, n_cells(h->p), h->stream), "nn to fp32");
  h->have_losses = true;
  h->have_weights = true;
  return RSOL_OK;
}

int rsol_set_weights(rsol_handle h, void* w) {
  if (int rc = need(h, false, false)) return rc;
  if (int rc = sync_arrays(h)) return rc;
  h->cells_valid = false;  // the packets change (or the cell-list scratch is reused)
  if (!loss_layout(h->p)) return fail(h, RSOL_ESTATE, "handle created without RSOL_FLAG_WEIGHTS");
  if (!w && h->np > 0) return fail(h, RSOL_EINVAL, "NULL weight array");
  if (h->p.flags & RSOL_FLAG_TILED && !(h->p.flags & RSOL_FLAG_KEEP_ORDER))
    return fail(h, RSOL_EINVAL, "the tiled path does not carry packet weights");
  h->w = w;
  h->have_weights = true;
  return RSOL_OK;
}

int rsol_set_particles(rsol_handle h, void* pos, float* off, void* u, int32_t* id) {
  if (int rc = need(h, false, false)) return rc;
  h->cells_valid = false;  // new arrays: the lists and any packets they held are dropped
  h->arrays_stale = false;
  if (h->np > 0 && (!pos || !u || !id)) return fail(h, RSOL_EINVAL, "NULL packet pointer");
  if (fp32(h->p) && h->np > 0 && !off) return fail(h, RSOL_EINVAL, "FP32 form needs off");
  if (!fp32(h->p) && off) return fail(h, RSOL_EINVAL, "FP64 form takes no off array");
  h->pos = pos;
  h->off = off;
  h->u = u;
  h->id = id;
  h->have_packets = true;
  h->sorted_valid = false;
  h->steps_since_sort = 0;
  return RSOL_OK;
}

int rsol_positions_to_cells(rsol_handle h, const double* x, int32_t* cell, float* off) {
  if (int rc = need(h, false, false)) return rc;
  if (int rc = sync_arrays(h)) return rc;
  h->cells_valid = false;  // the packets change (or the cell-list scratch is reused)
  if (h->np == 0) return RSOL_OK;
  if (!x || !cell || !off) return fail(h, RSOL_EINVAL, "NULL pointer");
  RSOL_HIP(h, launch_positions_to_cells(x, cell, off, h->np, consts(h), h->stream), "positions_to_cells");
  return RSOL_OK;
}

int rsol_cells_to_positions(rsol_handle h, const int32_t* cell, const float* off, double* x) {
  if (int rc = need(h, false, false)) return rc;
  if (int rc = sync_arrays(h)) return rc;
  h->cells_valid = false;  // the packets change (or the cell-list scratch is reused)
  if (h->np == 0) return RSOL_OK;
  if (!x || !cell || !off) return fail(h, RSOL_EINVAL, "NULL pointer");
  RSOL_HIP(h, launch_cells_to_positions(cell, off, x, h->np, consts(h), h->stream), "cells_to_positions");
  return RSOL_OK;
}

int rsol_courant_dt(rsol_handle h, double* dt) {
  if (int rc = need(h, true, true)) return rc;
  if (int rc = sync_arrays(h)) return rc;  // reads the registered packets
  if (!dt) return fail(h, RSOL_EINVAL, "dt is NULL");
  if (h->np == 0) return fail(h, RSOL_EINVAL, "no packets");
  if (fp32(h->p)) {
    RSOL_HIP(h, launch_dt_inputs<float>(caller_packets<float>(h), h->B, h->have_losses ? h->nn : nullptr,
                                        (int)n_cells(h->p), h->red, h->stream),
             "dt inputs");
  } else {
    RSOL_HIP(h, launch_dt_inputs<double>(caller_packets<double>(h), h->B, h->have_losses ? h->nn : nullptr,
                                         (int)n_cells(h->p), h->red, h->stream),
             "dt inputs");
  }
  unsigned long long bits[4];
  RSOL_HIP(h, hipMemcpyAsync(bits, h->red, sizeof(bits), hipMemcpyDeviceToHost, h->stream), "dt copy");
  RSOL_HIP(h, hipStreamSynchronize(h->stream), "dt sync");
  double v[4];
  memcpy(v, bits, sizeof(v));
  const double beta_max = v[0], gamma_min = v[1], b_max = v[2], nn_max = v[3];
  const rsol_params& p = h->p;
  double lim = INFINITY;
  if (beta_max > 0) lim = fmin(lim, p.courant * p.dx / (p.c_tilde * beta_max));
  const double omega = (naive(p) ? 1.0 : p.c_tilde / p.c) * fabs(p.qomc) * b_max / gamma_min;
  if (omega > 0) lim = fmin(lim, p.courant / omega);
  // catastrophic losses (Sec. 4): dt < C N/|dN/dt| with the rate (c_tilde/c) sigma c beta n_n
  const double lrate = (p.c_tilde / p.c) * h->sigma * p.c * beta_max * nn_max;
  if (h->have_losses && lrate > 0) lim = fmin(lim, p.courant / lrate);
  if (!isfinite(lim)) return fail(h, RSOL_EINVAL, "timestep unbounded (no motion and no field)");
  *dt = lim;
  return RSOL_OK;
}

int rsol_set_dt(rsol_handle h, double dt) {
  if (int rc = need(h, false, false)) return rc;
  if (!(dt > 0) || !isfinite(dt)) return fail(h, RSOL_EINVAL, "dt must be finite and > 0");
  h->p.dt = dt;
  return RSOL_OK;
}

int rsol_get_dt(rsol_handle h, double* dt) {
  if (int rc = need(h, false, false)) return rc;
  if (!dt) return fail(h, RSOL_EINVAL, "dt is NULL");
  if (!(h->p.dt > 0)) {
    double c = 0.0;
    if (int rc = rsol_courant_dt(h, &c)) return rc;
    h->p.dt = c;
  }
  *dt = h->p.dt;
  return RSOL_OK;
}

int rsol_gather(rsol_handle h, void* Ep, void* Bp) {
  if (int rc = need(h, true, true)) return rc;
  if (int rc = sync_arrays(h)) return rc;  // reads the registered packets
  if (h->have_weights)
    return fail(h, RSOL_EINVAL, "weights or losses registered: the separate phases carry neither (use rsol_step)");
  if (h->np == 0) return RSOL_OK;
  if (!Ep || !Bp) return fail(h, RSOL_EINVAL, "NULL output");
  if (fp32(h->p))
    RSOL_HIP(h, launch_gather<float>(h->p.shape, caller_packets<float>(h), h->E32, h->B32, (float*)Ep, (float*)Bp,
                                     consts(h), h->stream), "gather");
  else
    RSOL_HIP(h, launch_gather<double>(h->p.shape, caller_packets<double>(h), h->E, h->B, (double*)Ep, (double*)Bp,
                                      consts(h), h->stream), "gather");
  return RSOL_OK;
}

int rsol_push(rsol_handle h, const void* Ep, const void* Bp, void* payload) {
  if (int rc = need(h, false, true)) return rc;
  if (int rc = sync_arrays(h)) return rc;
  h->cells_valid = false;  // the packets change (or the cell-list scratch is reused)
  if (h->have_weights)
    return fail(h, RSOL_EINVAL, "weights or losses registered: the separate phases carry neither (use rsol_step)");
  if (h->np == 0) return RSOL_OK;
  if (!Ep || !Bp || !payload) return fail(h, RSOL_EINVAL, "NULL pointer");
  if (!(h->p.dt > 0)) return fail(h, RSOL_ESTATE, "dt not set");
  if (fp32(h->p))
    RSOL_HIP(h, launch_push<float>(caller_packets<float>(h), (const float*)Ep, (const float*)Bp, (float*)payload,
                                   consts(h), h->stream), "push");
  else
    RSOL_HIP(h, launch_push<double>(caller_packets<double>(h), (const double*)Ep, (const double*)Bp,
                                    (double*)payload, consts(h), h->stream), "push");
  return RSOL_OK;
}

int rsol_deposit(rsol_handle h, const void* payload, double* dM, double* dE) {
  if (int rc = need(h, false, true)) return rc;
  if (int rc = sync_arrays(h)) return rc;  // reads the registered packets
  if (h->have_weights)
    return fail(h, RSOL_EINVAL, "weights or losses registered: the separate phases carry neither (use rsol_step)");
  if (h->np == 0) return RSOL_OK;
  if (!payload || !dM) return fail(h, RSOL_EINVAL, "NULL pointer");
  if (fp32(h->p))
    RSOL_HIP(h, launch_deposit<float>(h->p.shape, caller_packets<float>(h), (const float*)payload, dM, dE, consts(h),
                                      h->stream), "deposit");
  else
    RSOL_HIP(h, launch_deposit<double>(h->p.shape, caller_packets<double>(h), (const double*)payload, dM, dE,
                                       consts(h), h->stream), "deposit");
  return RSOL_OK;
}

int rsol_drift(rsol_handle h) {
  if (int rc = need(h, false, true)) return rc;
  if (int rc = sync_arrays(h)) return rc;
  h->cells_valid = false;  // the packets change (or the cell-list scratch is reused)
  if (h->have_weights)
    return fail(h, RSOL_EINVAL, "weights or losses registered: the separate phases carry neither (use rsol_step)");
  if (h->np == 0) return RSOL_OK;
  if (!(h->p.dt > 0)) return fail(h, RSOL_ESTATE, "dt not set");
  if (fp32(h->p))
    RSOL_HIP(h, launch_drift<float>(caller_packets<float>(h), consts(h), h->stream), "drift");
  else
    RSOL_HIP(h, launch_drift<double>(caller_packets<double>(h), consts(h), h->stream), "drift");
  h->sorted_valid = false;
  return RSOL_OK;
}

int rsol_sort(rsol_handle h) {
  if (int rc = need(h, false, true)) return rc;
  if (int rc = sync_arrays(h)) return rc;
  h->cells_valid = false;  // the packets change (or the cell-list scratch is reused)
  if (h->have_weights) return fail(h, RSOL_EINVAL, "weights or losses registered: packets are re-binned by rsol_step only");
  return fp32(h->p) ? do_sort<float>(h, true) : do_sort<double>(h, true);
}

int rsol_step(rsol_handle h, int32_t nsteps, double* dM, double* dE) {
  if (int rc = need(h, true, true)) return rc;
  if (int rc = losses_path_ok(h)) return rc;
  if (nsteps < 0) return fail(h, RSOL_EINVAL, "nsteps < 0");
  if (!(h->p.dt > 0)) return fail(h, RSOL_ESTATE, "dt not set");
  if (!dM && dE) return fail(h, RSOL_EINVAL, "dE without dM");
  if (h->np == 0 || nsteps == 0) return RSOL_OK;
  const GasLink none{};
  return fp32(h->p) ? do_step<float>(h, nsteps, dM, dE, none) : do_step<double>(h, nsteps, dM, dE, none);
}

int rsol_step_coupled(rsol_handle h, int32_t nsteps, const double* rho, double* mom, double* egas, double* E) {
  if (int rc = need(h, true, true)) return rc;
  if (int rc = losses_path_ok(h)) return rc;
  if (nsteps < 0) return fail(h, RSOL_EINVAL, "nsteps < 0");
  if (!(h->p.dt > 0)) return fail(h, RSOL_ESTATE, "dt not set");
  if (!rho || !mom || !E) return fail(h, RSOL_EINVAL, "NULL gas pointer");
  const double* Ec = E;
  if (Ec == h->B || Ec == rho || E == mom || (egas && (E == egas || egas == mom)))
    return fail(h, RSOL_EINVAL, "gas arrays alias each other or B");
  GasLink g{};
  g.rho = rho;
  g.mom = mom;
  g.egas = egas;
  g.B = h->B;
  g.E = E;
  g.E32 = fp32(h->p) ? h->E32 : nullptr;
  g.inv_c = 1.0 / h->p.c;
  h->E = E;
  RSOL_HIP(h, launch_gas_field(g, n_cells(h->p), h->stream), "gas field");
  if (h->np == 0 || nsteps == 0) return RSOL_OK;
  return fp32(h->p) ? do_step<float>(h, nsteps, mom, egas, g) : do_step<double>(h, nsteps, mom, egas, g);
}

int rsol_sync_particles(rsol_handle h) {
  if (int rc = need(h, false, false)) return rc;
  return sync_arrays(h);
}

int rsol_moments(rsol_handle h, double* rho, double* P, double* e) {
  if (int rc = need(h, false, true)) return rc;
  if (int rc = sync_arrays(h)) return rc;  // reads the registered packets
  const int64_t nc = n_cells(h->p);
  if (rho) RSOL_HIP(h, launch_fill_f64(rho, 0.0, nc, h->stream), "zero rho");
  if (P) RSOL_HIP(h, launch_fill_f64(P, 0.0, 3 * nc, h->stream), "zero P");
  if (e) RSOL_HIP(h, launch_fill_f64(e, 0.0, nc, h->stream), "zero e");
  if (h->np == 0) return RSOL_OK;
  if (fp32(h->p)) return moments<float>(h, rho, P, e);
  return moments<double>(h, rho, P, e);
}

int rsol_set_flags(rsol_handle h, int32_t flags) {
  if (int rc = need(h, false, false)) return rc;
  if (int rc = sync_arrays(h)) return rc;
  h->cells_valid = false;  // the packets change (or the cell-list scratch is reused)
  if (flags & ~kKnownFlags) return fail(h, RSOL_EINVAL, "unknown flag bits");
  if (!flag_conflict(flags).empty()) return fail(h, RSOL_EINVAL, flag_conflict(flags));
  if ((flags ^ h->p.flags) & RSOL_FLAG_LOSSES) return fail(h, RSOL_EINVAL, "RSOL_FLAG_LOSSES is fixed at rsol_init");
  if (h->have_weights && (flags & RSOL_FLAG_TILED) && !(flags & RSOL_FLAG_KEEP_ORDER))
    return fail(h, RSOL_EINVAL, "the tiled path does not carry losses");
  h->p.flags = flags;
  return RSOL_OK;
}

size_t rsol_state_bytes(rsol_handle h) {
  if (!h) return 0;
  return slab_layout(h).total;
}

int rsol_record_states(rsol_handle h, int32_t nsteps, void* states) {
  if (int rc = need(h, true, true)) return rc;
  if (int rc = sync_arrays(h)) return rc;
  h->cells_valid = false;  // the packets change (or the cell-list scratch is reused)
  if (naive(h->p)) return fail(h, RSOL_EINVAL, "the differentiation form covers the RSOL equations only");
  if (pusher_of(h->p.flags) != kPushBoris) return fail(h, RSOL_EINVAL, "the differentiation form is the Boris pusher's");
  if (h->have_weights) return fail(h, RSOL_EINVAL, "the differentiation form carries no packet weights or losses");
  if (nsteps < 0) return fail(h, RSOL_EINVAL, "nsteps < 0");
  if (!(h->p.dt > 0)) return fail(h, RSOL_ESTATE, "dt not set");
  if (h->np == 0 || nsteps == 0) return RSOL_OK;
  if (!states) return fail(h, RSOL_EINVAL, "states is NULL");
  const RunConsts k = consts(h);
  h->sorted_valid = false;
  if (fp32(h->p)) return adj_tiled(h) ? record_tiled<float>(h, nsteps, (char*)states, k)
                                      : record_global<float>(h, nsteps, (char*)states, k);
  return adj_tiled(h) ? record_tiled<double>(h, nsteps, (char*)states, k)
                      : record_global<double>(h, nsteps, (char*)states, k);
}

int rsol_step_backward(rsol_handle h, int32_t nsteps, const void* states, void* lam_x, void* lam_u,
                       const double* lam_dM, const double* lam_dE, double* gE, double* gB) {
  if (int rc = need(h, true, true)) return rc;
  if (int rc = sync_arrays(h)) return rc;
  h->cells_valid = false;  // the packets change (or the cell-list scratch is reused)
  if (naive(h->p)) return fail(h, RSOL_EINVAL, "the differentiation form covers the RSOL equations only");
  if (pusher_of(h->p.flags) != kPushBoris) return fail(h, RSOL_EINVAL, "the differentiation form is the Boris pusher's");
  if (h->have_weights) return fail(h, RSOL_EINVAL, "the differentiation form carries no packet weights or losses");
  if (nsteps < 0) return fail(h, RSOL_EINVAL, "nsteps < 0");
  if (!(h->p.dt > 0)) return fail(h, RSOL_ESTATE, "dt not set");
  if (!lam_dM && lam_dE) return fail(h, RSOL_EINVAL, "lam_dE without lam_dM");
  if (h->np == 0 || nsteps == 0) return RSOL_OK;
  if (!states || !lam_x || !lam_u || !gE || !gB) return fail(h, RSOL_EINVAL, "NULL pointer");
  const RunConsts k = consts(h);
  h->sorted_valid = false;
  if (fp32(h->p))
    return adj_tiled(h) ? backward_tiled<float>(h, nsteps, (const char*)states, (float*)lam_x, (float*)lam_u, lam_dM,
                                                lam_dE, gE, gB, k)
                        : backward_global<float>(h, nsteps, (const char*)states, (float*)lam_x, (float*)lam_u, lam_dM,
                                                 lam_dE, gE, gB, k);
  return adj_tiled(h) ? backward_tiled<double>(h, nsteps, (const char*)states, (double*)lam_x, (double*)lam_u, lam_dM,
                                               lam_dE, gE, gB, k)
                      : backward_global<double>(h, nsteps, (const char*)states, (double*)lam_x, (double*)lam_u, lam_dM,
                                                lam_dE, gE, gB, k);
}

int rsol_moments_backward(rsol_handle h, const double* lam_rho, const double* lam_P, const double* lam_e,
                          void* lam_x, void* lam_u) {
  if (int rc = need(h, false, true)) return rc;
  if (int rc = sync_arrays(h)) return rc;  // reads the registered packets
  if (naive(h->p)) return fail(h, RSOL_EINVAL, "the differentiation form covers the RSOL equations only");
  if (pusher_of(h->p.flags) != kPushBoris) return fail(h, RSOL_EINVAL, "the differentiation form is the Boris pusher's");
  if (h->have_weights) return fail(h, RSOL_EINVAL, "the differentiation form carries no packet weights or losses");
  if (h->np == 0) return RSOL_OK;
  if (!lam_x || !lam_u) return fail(h, RSOL_EINVAL, "NULL adjoint array");
  if (fp32(h->p))
    RSOL_HIP(h, launch_moments_backward<float>(h->p.shape, caller_packets<float>(h), lam_rho, lam_P, lam_e,
                                               (float*)lam_x, (float*)lam_u, consts(h), h->stream), "moments backward");
  else
    RSOL_HIP(h, launch_moments_backward<double>(h->p.shape, caller_packets<double>(h), lam_rho, lam_P, lam_e,
                                                (double*)lam_x, (double*)lam_u, consts(h), h->stream),
             "moments backward");
  return RSOL_OK;
}

int rsol_stray_count(rsol_handle h, int64_t* n) {
  if (int rc = need(h, false, false)) return rc;
  if (!n) return fail(h, RSOL_EINVAL, "n is NULL");
  uint32_t word = 0;
  RSOL_HIP(h, hipMemcpyAsync(&word, h->status + 1, sizeof(word), hipMemcpyDeviceToHost, h->stream), "stray copy");
  RSOL_HIP(h, hipStreamSynchronize(h->stream), "stray sync");
  RSOL_HIP(h, launch_fill_u32(h->status + 1, 0u, 1, h->stream), "stray clear");
  *n = word;
  return RSOL_OK;
}

int rsol_check(rsol_handle h) {
  if (int rc = need(h, false, false)) return rc;
  uint32_t word = 0;
  RSOL_HIP(h, hipMemcpyAsync(&word, h->status, sizeof(word), hipMemcpyDeviceToHost, h->stream), "status copy");
  RSOL_HIP(h, hipStreamSynchronize(h->stream), "status sync");
  RSOL_HIP(h, launch_fill_u32(h->status, 0u, 1, h->stream), "status clear");
  if (word & ERR_NAN) return fail(h, RSOL_ENAN, "non-finite packet momentum");
  if (word & ERR_TILE) return fail(h, RSOL_ETILE, "a packet left its tile's staged region between re-sorts (tiled path) or the cell lists overflowed");
  if (word & ERR_COURANT) return fail(h, RSOL_ECOURANT, "a packet moved further than the per-step bound");
  return RSOL_OK;
}

}  // extern "C"
