/*
 * rsol.h -- C ABI of the MI355X (gfx950) library for the data-parallel hot path
 * of the reduced-speed-of-light (RSOL) MHD particle-in-cell method of
 * Ji & Hopkins, "A Reduced-Speed-of-Light Formulation of the MHD-PIC Method"
 * (arXiv:2111.14704).
 *
 * Per packet step (Sec. 2):
 *   gather   E_p, B_p = sum_i W(x_p - x_i) (E_i, B_i)                  kernel W of Eq. (4)
 *   kick     d(gamma beta)/dt = (c_tilde/c) (q/(m c)) [E + beta x B]     Eq. (11)
 *   exchange d(rho u)/dt = -sum_j (1/V_j)(c/c_tilde) d_t P_j             Eq. (12)
 *   drift    d<x>/dt = (c_tilde/c) <v> = c_tilde beta                   Sec. 2
 * with E = -(u/c) x B from the gas velocity u and the TRUE c (Sec. 2, after Eq. (5)),
 * gamma and beta the packet's true values (Eqs. (7)-(8)), P_j = M_j c u_j and
 * energy M_j c^2 gamma_j (Eqs. (9)-(10)).  The integrator is the relativistic
 * Boris scheme, leapfrog in time: the state is (x^n, u^{n-1/2}).
 *
 * Conventions shared by every entry point
 *  - Grid: periodic, nx*ny*nz cells of side dx, cell-centred collocated fields.
 *    Grid arrays are [C][n_cells] doubles, cell = ix + nx*(iy + ny*iz) (x fastest).
 *  - Packets: structure of arrays over np packets.
 *      FP64 form: x[3][np] absolute positions (double, in [0, L)), u[3][np] (double)
 *      FP32 form: cell[np] home cell (int32), off[3][np] in-cell offset in cells
 *                 (float, in [0, 1)), u[3][np] (float)
 *    u = gamma*beta, the packet momentum in units of m c; id[np] (int32) labels packets.
 *    With RSOL_FLAG_RESIDENT the packets live in the library's cell lists between steps
 *    and the registered arrays are current only after rsol_sync_particles (or any
 *    entry point that reads them).
 *  - Every pointer argument is a DEVICE pointer owned by the caller unless stated.
 *    The library never allocates or frees device memory; it keeps the pointers given
 *    to rsol_init / rsol_set_* until rsol_destroy.
 *  - All work is enqueued on the stream given to rsol_init and is asynchronous;
 *    only rsol_courant_dt, rsol_check, rsol_stray_count and rsol_timing_read
 *    synchronise that stream.
 *  - Every call returns RSOL_OK (0) or a negative status; rsol_last_error gives the
 *    message.  No C++ exception crosses this boundary.
 *  - Calls on one handle must not overlap from several host threads.
 */
#ifndef RSOL_H
#define RSOL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum rsol_status {
  RSOL_OK = 0,
  RSOL_EINVAL = -1,   /* bad argument (NULL pointer, size, parameter out of range)          */
  RSOL_ESTATE = -2,   /* call out of order (fields or packets not registered yet)           */
  RSOL_EHIP = -3,     /* a HIP runtime call or kernel launch failed                          */
  RSOL_ECOURANT = -4, /* a packet moved further in one step than the configured bound       */
  RSOL_ENAN = -5,     /* a non-finite momentum appeared                                      */
  RSOL_ESCRATCH = -6, /* scratch buffer smaller than rsol_scratch_bytes()                    */
  RSOL_ETILE = -7     /* a packet left the region staged for its tile between re-sorts      */
};

enum rsol_shape { RSOL_CIC = 1, RSOL_TSC = 2 };   /* cloud-in-cell / triangular-shaped cloud */
enum rsol_precision { RSOL_FP64 = 0, RSOL_FP32 = 1 };

typedef struct rsol_params {
  int32_t nx, ny, nz;   /* grid cells per axis, each 1..1024                                  */
  int32_t shape;        /* RSOL_CIC or RSOL_TSC: the spatial kernel W of Eq. (4)              */
  int32_t precision;    /* RSOL_FP64 or RSOL_FP32 (packet state and push arithmetic)          */
  int32_t sort_every;   /* re-bin packets by cell every K steps inside rsol_step (1..8)      */
  int32_t flags;        /* RSOL_FLAG_* bits                                                   */
  int32_t reserved;     /* must be 0                                                          */
  double dx;            /* cell size (V = dx^3)                                               */
  double c;             /* true speed of light                                                */
  double c_tilde;       /* reduced speed of light, 0 < c_tilde <= c                           */
  double qomc;          /* q / (m_s c) of the CR species                                      */
  double dt;            /* timestep; may be 0 until rsol_set_dt                                */
  double courant;       /* Courant factor C of Sec. 4 (0 < C <= 0.5)                          */
  double mass;          /* packet mass weight M_j = N_j <m_s> (times w_j with rsol_set_weights) */
} rsol_params;

/* flags */
#define RSOL_FLAG_KEEP_ORDER 1  /* rsol_step keeps the packet order (never re-bins) and runs the
                                   one-thread-per-packet kernel with global atomics.  When
                                   dM and dE are both NULL (the differentiation form's forward
                                   pass), with the Boris pusher and no losses, the steps run
                                   instead on a scratch copy sorted by tile every four steps,
                                   with each tile's E and B staged on chip (the same
                                   arithmetic in the same order); the caller's arrays end in
                                   their own order either way                                 */
#define RSOL_FLAG_TILED 2       /* rsol_step runs the tiled LDS kernel over packets re-sorted
                                   every sort_every steps instead of the default cell-list
                                   kernel (ignored under RSOL_FLAG_KEEP_ORDER).  The tiles of
                                   this path and of the differentiation form are 4x4x4 cells;
                                   the environment variable RSOL_TILE="tx,ty,tz" (read when a
                                   handle is created or sized) sets another shape, with
                                   tx*ty*tz <= 256                                           */
#define RSOL_FLAG_NAIVE 4       /* contrast mode: the naive substitution of c by c_tilde that
                                   the RSOL formulation replaces (Sec. 1; Sec. 5, items (1)-(4)).
                                   u = gamma v / c_tilde with du/dt = (q/(m c)) [(c/c_tilde) E +
                                   beta x B] (the momentum equation of Sec. 5, item (3)); packet
                                   momentum M c_tilde u and energy M c_tilde^2 gamma in the
                                   exchange and the moments, no c/c_tilde on the back-reaction;
                                   rsol_courant_dt's gyro limit uses the unreduced q|B|/(gamma m c).
                                   Drift, E and every kernel are the RSOL ones; the
                                   differentiation-form entry points return RSOL_EINVAL.      */
#define RSOL_FLAG_LOSSES 8      /* set at rsol_init: the scratch layout carries a weight per
                                   packet so that rsol_set_weights can register per-packet
                                   weights and rsol_set_losses switch on catastrophic losses;
                                   fixed for the life of the handle                           */
#define RSOL_FLAG_WEIGHTS 8     /* the same bit, named for per-packet weights alone           */
#define RSOL_FLAG_PUSHER_VAY 16 /* momentum update by the pusher of Vay (Phys. Plasmas 15,
                                   056701, 2008) instead of Boris, for the same Eq. (11) and
                                   the same half kicks; keeps the force-free E x B drift
                                   exactly.  Cell-list and keep-order paths and rsol_push; the
                                   tiled path and the differentiation form refuse it.        */
#define RSOL_FLAG_PUSHER_HC 32  /* the same with the pusher of Higuera and Cary (Phys. Plasmas
                                   24, 052104, 2017); at most one pusher flag.               */
#define RSOL_FLAG_RESIDENT 64   /* default (cell-list) path: the packets stay in the
                                   library's cell lists between rsol_step / rsol_step_coupled
                                   calls, which then neither file the registered arrays nor
                                   copy the packets back.  The arrays are brought up to date
                                   by rsol_sync_particles, and by every other entry point
                                   that reads or writes them, before it does; entry points
                                   that change the packets (rsol_set_particles,
                                   rsol_set_losses, rsol_set_flags, rsol_sort, rsol_push,
                                   rsol_drift, the other step paths, the differentiation
                                   form, the position conversions) also drop the lists, and
                                   the next call files again.  While the flag is set the
                                   caller reads the arrays only after rsol_sync_particles
                                   and writes them only followed by rsol_set_particles     */
#define RSOL_FLAG_RECORD_ONLY 128 /* rsol_record_states records the states but leaves the
                                   caller's packet arrays as it found them (the recorded
                                   states are the same); for a reverse sweep that restores its
                                   own checkpoints before each recording.                   */

typedef struct rsol_ctx* rsol_handle;

/* Bytes of device scratch rsol_init needs for these parameters and np packets; 0 when
 * the default path's cell lists cannot hold them (their id and weight arrays, up to 8
 * bytes per slot, are addressed by 32-bit byte offsets: at most 512M slots, about 100
 * packets per cell on a 128^3 grid). */
size_t rsol_scratch_bytes(const rsol_params* p, int64_t n_particles);

/* Create a handle.  p is copied (host pointer).  stream: a hipStream_t (NULL = default
 * stream).  scratch: caller-owned device buffer of at least rsol_scratch_bytes() bytes,
 * 256-byte aligned, kept until rsol_destroy.  Errors: RSOL_EINVAL for out-of-range
 * parameters or too many packets for the cell lists, RSOL_ESCRATCH if scratch_bytes is
 * too small. */
int rsol_init(const rsol_params* p, int64_t n_particles, void* stream, void* scratch,
              size_t scratch_bytes, rsol_handle* out);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): one call that does what rsol_init,
 * rsol_set_fields, rsol_set_particles, rsol_set_dt and rsol_step do together, with the
 * scratch taken from a static device array inside the library (64 MiB per GPU, held by
 * each GPU the library runs on until the process ends) instead of a caller buffer.
 * Nothing here allocates device memory.  Arguments as for those entry points: p with
 * p->dt > 0 (no Courant timestep is computed here) and neither RSOL_FLAG_RESIDENT nor
 * RSOL_FLAG_LOSSES; E, B [3][n_cells] doubles; pos/off/u/id the packet arrays of the
 * precision (updated in place, permuted as rsol_step permutes them); dM, dE added to as
 * rsol_step adds (both may be NULL; dE needs dM).  The stream must belong to the current
 * device.  Errors: RSOL_ESCRATCH when rsol_scratch_bytes(p, n_particles) exceeds the
 * static array, the other codes as rsol_init and rsol_step; the message is
 * rsol_last_error(NULL).  Device-detected faults (RSOL_ECOURANT, RSOL_ENAN) are not
 * reported (there is no handle to check).  All calls on one GPU share its array, which
 * keeps the last call's contents: calls that overlap on one GPU (several host threads,
 * or work still running on another stream) race and corrupt each other. */
int rsol_step_static(const rsol_params* p, int64_t n_particles, void* stream, const double* E, const double* B,
                     void* pos, float* off, void* u, int32_t* id, int32_t nsteps, double* dM, double* dE);

/* Free the host-side handle (device memory stays with the caller). */
int rsol_destroy(rsol_handle h);

/* Message of the last failure on h (or of the last failed rsol_init when h is NULL).
 * The string is owned by the library and valid until the next call on h. */
const char* rsol_last_error(rsol_handle h);

/* E = -(u_gas/c) x B at every cell centre with the true c (Sec. 2, after Eq. (5)).
 * u_gas, B: [3][n_cells] in; E: [3][n_cells] out (may not alias the inputs). */
int rsol_electric_field(rsol_handle h, const double* u_gas, const double* B, double* E);

/* Register the grid fields E, B ([3][n_cells] doubles) used by the gather.  The
 * FP32 form takes float copies into scratch here, so call again after changing them. */
int rsol_set_fields(rsol_handle h, const double* E, const double* B);

/* Catastrophic losses (Sec. 2, collisional terms; Sec. 4 for the timestep).  Every
 * packet total (N, M, energy, P) decays at the reduced rate (c_tilde/c) <sigma v> n_n with
 * <sigma v> = sigma c beta, beta from the packet's momentum after the kick and n_n the
 * nucleon density gathered at the packet's position before the drift with the kernel W;
 * the decay over a step is integrated exactly with that frozen rate.  The exchange
 * deposit becomes the change of the weighted packet totals, so what the losses remove
 * goes to the gas with the same -(c/c_tilde) factor (Eq. (12)).
 *   sigma  cross-section (area in the units of dx^2), >= 0
 *   nn     [n_cells] nucleon number density (doubles); read by every later step (the
 *          FP32 form takes a float copy here, so call again after changing it)
 *   w      [np] packet weights N_j/N (precision type), in/out: updated by rsol_step and
 *          rsol_step_coupled and permuted with the packets; the moments weight by it.
 * Needs a handle created with RSOL_FLAG_LOSSES (else RSOL_ESTATE).  Supported by the
 * default cell-list path and RSOL_FLAG_KEEP_ORDER; with losses registered, the tiled
 * path, rsol_sort, the separate phases (gather/push/deposit/drift) and the
 * differentiation form return RSOL_EINVAL.  rsol_courant_dt adds the limit
 * dt < C / ((c_tilde/c) sigma c beta_max n_n,max). */
int rsol_set_losses(rsol_handle h, double sigma, const double* nn, void* w);

/* Per-packet weights (Sec. 2, Eq. (4): a packet stands for N_j particles; Sec. 4 sets
 * N_j from the total mass or energy): the packet mass becomes M_j = mass * w_j for the
 * exchange of Eq. (12) and for the moments.  w: [np] weights in the precision type,
 * device pointer, kept until rsol_destroy and permuted with the packets by rsol_step
 * (rsol_set_losses registers the same array, and makes the weights decay).  Needs a
 * handle created with RSOL_FLAG_WEIGHTS (else RSOL_ESTATE).  Honoured by the default
 * cell-list path, RSOL_FLAG_KEEP_ORDER and rsol_moments; with weights registered the
 * tiled path, rsol_sort, the separate phases and the differentiation form return
 * RSOL_EINVAL. */
int rsol_set_weights(rsol_handle h, void* w);

/* Register the packet state (Sec. 2, Eq. (4): packets {x, p} with weights N_j).
 * FP64 form: pos = double x[3][np], off = NULL, u = double[3][np].
 * FP32 form: pos = int32 cell[np], off = float[3][np], u = float[3][np].
 * id: int32[np].  The arrays are updated in place by push/drift/step and permuted
 * (with id) by rsol_sort and rsol_step. */
int rsol_set_particles(rsol_handle h, void* pos, float* off, void* u, int32_t* id);

/* Precision-form position conversions: absolute x[3][np] (double) <-> home cell[np]
 * (int32) + in-cell offset off[3][np] (float).  np is the handle's packet count. */
int rsol_positions_to_cells(rsol_handle h, const double* x, int32_t* cell, float* off);
int rsol_cells_to_positions(rsol_handle h, const int32_t* cell, const float* off, double* x);

/* RSOL Courant timestep (Sec. 4): dt = C min(dx/(c_tilde max beta), 1/Omega_eff,max) with
 * Omega_eff = (c_tilde/c) qomc |B| / gamma, from the registered packets (max beta, min
 * gamma) and fields (max |B|).  Synchronises the stream; *dt is a host pointer.  Does
 * not change the handle's dt (use rsol_set_dt). */
int rsol_courant_dt(rsol_handle h, double* dt);
int rsol_set_dt(rsol_handle h, double dt);
/* The timestep the next step uses (Sec. 4): the handle's dt when set (rsol_params.dt > 0
 * or rsol_set_dt); when it is 0, the Courant timestep of the registered packets and
 * fields (rsol_courant_dt) becomes the handle's dt and is returned.  *dt is a host
 * pointer.  RSOL_ESTATE when dt is unset and fields or packets are not registered. */
int rsol_get_dt(rsol_handle h, double* dt);

/* A packet step split into its phases, for any packet order.
 * rsol_gather: Ep, Bp [3][np] (precision type) = fields at the current positions.
 * rsol_push:   u <- u^{n+1/2} from Ep, Bp (Eq. (11)); payload [4][np] (precision type)
 *              = (du_x, du_y, du_z, dgamma) of the step.
 * rsol_deposit: adds -(c/c_tilde) M c du W / V to dM[3][n_cells] and -(c/c_tilde) M c^2
 *              dgamma W / V to dE[n_cells] (Eq. (12)) with W at the CURRENT positions,
 *              i.e. call before rsol_drift; dE may be NULL.
 * rsol_drift:  x <- x + c_tilde dt u/gamma with periodic wrap (Sec. 2, v_eff = c_tilde beta). */
int rsol_gather(rsol_handle h, void* Ep, void* Bp);
int rsol_push(rsol_handle h, const void* Ep, const void* Bp, void* payload);
int rsol_deposit(rsol_handle h, const void* payload, double* dM, double* dE);
int rsol_drift(rsol_handle h);

/* Counting sort of the packets by tile-major home cell (build-internal ordering; the
 * registered arrays are permuted in place, id with them). */
int rsol_sort(rsol_handle h);

/* nsteps fused packet steps (gather, kick, exchange deposit at x^n, drift).  The
 * exchange of every step is ADDED to dM[3][n_cells] and dE[n_cells] (dM NULL skips the
 * deposit; dE may be NULL).  Default path: the packets are filed into per-cell buckets
 * in scratch, every step moves each packet into the bucket of its new cell, and on
 * return the registered arrays hold the packets in cell-major order (id permuted with
 * them).  RSOL_FLAG_TILED: re-sort every sort_every steps and run the tiled kernel.
 * RSOL_FLAG_KEEP_ORDER: packet order unchanged. */
int rsol_step(rsol_handle h, int32_t nsteps, double* dM, double* dE);

/* nsteps packet steps coupled to a gas whose density and magnetic field are held
 * fixed (no MHD solver).  Every step gathers E = -(u_gas/c) x B built from the gas
 * velocity u_gas = mom/rho with the true c (Sec. 2, after Eq. (5)); the step's exchange
 * is added into the gas, mom += dM and egas += dE (Eq. (12) and the same rule for the
 * packet energy of Eq. (9)), and E is rebuilt from the new mom before the next step.
 * The sums V sum mom + (c/c_tilde) sum_j M c u_j and V sum egas + (c/c_tilde) sum_j
 * M c^2 gamma_j are conserved up to rounding (Sec. 2, discussion after Eq. (12)).
 *   rho  [n_cells]     gas density (> 0), in
 *   mom  [3][n_cells]  gas momentum density rho u, in/out
 *   egas [n_cells]     gas energy density, in/out (NULL: not tracked)
 *   E    [3][n_cells]  out: on return the field of the final gas state.  E becomes the
 *                      handle's registered electric field (in place of the one given
 *                      to rsol_set_fields); B stays the registered one.
 * dt stays the handle's.  Packet order and paths follow rsol_step and its flags.
 * Errors: RSOL_EINVAL for NULL rho/mom/E or arrays that alias each other or B,
 * RSOL_ESTATE before fields, packets and dt are set; step errors as rsol_step. */
int rsol_step_coupled(rsol_handle h, int32_t nsteps, const double* rho, double* mom, double* egas, double* E);

/* Copy the packets held in resident cell lists (RSOL_FLAG_RESIDENT) back to the
 * registered arrays (cell-major order, ids permuted with them); a no-op when the arrays
 * are current.  Enqueued on the handle's stream. */
int rsol_sync_particles(rsol_handle h);

/* CR moments of the current state (Sec. 2 packet totals): rho[n_cells] = sum M W / V,
 * P[3][n_cells] = sum M c u W / V, e[n_cells] = sum M c^2 gamma W / V (times the packet
 * weight under losses).  Outputs are overwritten; any may be NULL.  The packets are
 * taken tile by tile (a sort of their indices in scratch; the registered arrays are not
 * touched) and summed per tile on chip, so the order of the additions into each cell
 * is not fixed: results agree to rounding from call to call. */
int rsol_moments(rsol_handle h, double* rho, double* P, double* e);

/* Set the RSOL_FLAG_* bits of the handle (RSOL_FLAG_LOSSES cannot change). */
int rsol_set_flags(rsol_handle h, int32_t flags);

/* ---- Differentiation form (reverse mode through gather -> push -> drift) ----
 * The adjoint of the deposit is a gather and the adjoint of the gather is a scatter.
 * Gradients flow to the grid fields E, B (as independent inputs) and to the initial
 * packet state; dt is a fixed parameter.  The adjoint arrays are in the order of the
 * caller's packet arrays at the time of recording (rsol_record_states leaves that order
 * as it found it). */

/* Bytes of one recorded step: the packet state (np * 48 in the FP64 form: x[3], u[3]
 * doubles; np * 28 in the FP32 form: cell, off[3], u[3] as 4-byte words) followed by the
 * tile ordering of its block of steps (np * 8 bytes plus 4 bytes per cell and one,
 * each part rounded up to 256 bytes).  The contents are internal to the library. */
size_t rsol_state_bytes(rsol_handle h);

/* Advance nsteps steps without exchange deposit, writing the state BEFORE each step
 * into states[n] (device buffer of nsteps * rsol_state_bytes).  The caller's packet
 * arrays end advanced by nsteps steps, in their own order (with RSOL_FLAG_RECORD_ONLY
 * they are left unchanged).  Internally the packets are
 * counting-sorted by tile every few steps into a scratch copy, which the steps advance
 * with each tile's E and B staged in on-chip memory; the recorded states are kept in
 * those orders, so that the reverse sweep reads them contiguously. */
int rsol_record_states(rsol_handle h, int32_t nsteps, void* states);

/* Reverse of the nsteps steps recorded in states by one rsol_record_states call (its
 * first nsteps steps), from step nsteps-1 down to 0.  Internally the adjoints are held
 * in the recorded tile orders, so that dL/dE and dL/dB accumulate in on-chip memory;
 * the caller's arrays keep their order.
 * lam_x, lam_u: [3][np] (precision type), on entry dL/d(x, u) after the last step, on
 * exit dL/d(x, u) before the first.  lam_dM [3][n_cells], lam_dE [n_cells]: cotangent of
 * the exchange summed over these steps (both may be NULL; lam_dE needs lam_dM).
 * gE, gB: [3][n_cells] doubles, ACCUMULATED (+=).  Device pointers. */
int rsol_step_backward(rsol_handle h, int32_t nsteps, const void* states, void* lam_x, void* lam_u,
                       const double* lam_dM, const double* lam_dE, double* gE, double* gB);

/* Adjoint of rsol_moments at the current state: adds to lam_x, lam_u ([3][np]) the
 * gradient of sum(lam_rho*rho) + sum(lam_P*P) + sum(lam_e*e); any cotangent may be NULL. */
int rsol_moments_backward(rsol_handle h, const double* lam_rho, const double* lam_P, const double* lam_e,
                          void* lam_x, void* lam_u);

/* Launch timing (a profiling aid, not part of the method): while enabled, every step and
 * sort launch made by rsol_step / rsol_sort is bracketed by HIP events on the handle's
 * stream, and so is every reverse-step launch of rsol_step_backward (counted with the
 * step launches).  rsol_timing_read synchronises the stream, returns the summed
 * milliseconds and launch counts since the last read (host pointers, any may be NULL)
 * and resets them. */
int rsol_timing(rsol_handle h, int32_t enable);
int rsol_timing_read(rsol_handle h, double* step_ms, int64_t* n_step, double* sort_ms, int64_t* n_sort);

/* Number of packet-steps since the last call that ran on the tiled kernel's fallback path
 * (stencil outside its tile's staged region, e.g. after a timestep above the Courant
 * limit).  Synchronises the stream; *n is a host pointer; the counter is cleared. */
int rsol_stray_count(rsol_handle h, int64_t* n);

/* Synchronise the stream and report device-detected faults since the last check:
 * RSOL_ECOURANT, RSOL_ENAN, RSOL_ETILE (the word is cleared). */
int rsol_check(rsol_handle h);

#ifdef __cplusplus
}
#endif

#endif /* RSOL_H */
