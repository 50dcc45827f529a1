#!/usr/bin/env python3
"""Throughput of the fused RSOL packet step on one MI355X.

A step is one pass of the whole hot path over every packet of the workload: the
cell-list fused kernel (gather E and B, relativistic Boris kick with the RSOL
factors, exchange deposit, drift, and the move of every packet into the store of
its new cell) plus the kernel that adds the per-tile exchange into the grid.  The
packets are filed into the cell lists once per rsol_step call and copied back to
the caller's arrays at its end; both are inside the timed region.  Inputs are
resident in HBM before the timed region; the timed region is exactly --steps steps
bracketed by device synchronisation.

Prints ONE JSON line.  The headline is workload 4 (128^3 cells x 32 packets per
cell, TSC, c/c_tilde = 100): value = particle-updates/s of the FP64 path (wall clock
over the timed steps); "fp32" = the precision form on the same workload, with its
speedup over FP64; "roofline" = the FP64 step kernel's algorithmic HBM bytes per
launch over its event-timed average duration against the 8 TB/s HBM3E peak;
"hbm_frac_full_step" (top level and in "fp32") = the metric's % of HBM peak, as a fraction, on the whole
step rate, i.e. algorithmic bytes per packet-step times the wall-clock rate;
"extras" = the same pair on workload 2 (64^3 x 64 ppc) and, on it, the FP64 step
coupled to the workload's gas ("coupled"), in the naive-substitution contrast mode
("naive"), with catastrophic losses ("losses"), with the Vay and Higuera-Cary
momentum updates ("pushers"), and one step per rsol_step call filing the packets
every call and with RSOL_FLAG_RESIDENT ("one_step_calls");
"backward" = the differentiation form on workload 5, with a roofline over the whole
backward pass (algorithmic bytes of the recompute and the reverse step per
packet-step); "copy_gbs" in each roofline = a plain device-to-device copy's measured
bandwidth on the same GPU, "frac_of_copy" the achieved bandwidth against it;
"cpu_baseline" = the CPU oracle timed on a bounded sample of the headline workload.
"""

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "particle-updates/s (gather+RSOL push+deposit), FP32 vs FP64, % of HBM peak"
KERNEL_SOURCES = ["paper_2111_14704_amd/csrc/kernels_cells.hip", "paper_2111_14704_amd/csrc/rsol_cells.hpp",
                  "paper_2111_14704_amd/csrc/rsol_device.hpp"]
REVERSE_SOURCES = ["paper_2111_14704_amd/csrc/kernels_adjoint.hip", "paper_2111_14704_amd/csrc/rsol_adjoint.hpp",
                   "paper_2111_14704_amd/csrc/rsol_particles.hpp", "paper_2111_14704_amd/csrc/rsol_device.hpp"]


def kernel_hash(sources=KERNEL_SOURCES):
    h = hashlib.sha256()
    for rel in sources:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def algorithmic_bytes_per_packet_step(precision, ppc):
    """Bytes one packet-step must move at minimum: the packet state read and written
    once, plus the grid fields read once and the exchange read-modify-written once per
    cell, shared by the ppc packets of a cell."""
    if precision == "fp64":
        packet = 2 * (3 * 8 + 3 * 8)           # x, u read + write
        cell = 6 * 8 + 2 * 4 * 8               # E, B read; dM (3) + dE read + write, FP64
    else:
        packet = 2 * (4 + 3 * 4 + 3 * 4)       # cell, offset, u read + write
        cell = 6 * 4 + 2 * 4 * 8               # FP32 E, B read; FP64 exchange read + write
    return packet + cell / ppc


def algorithmic_bytes_backward(precision, ppc):
    """Bytes one packet-step of the backward pass must move at minimum (checkpoints every
    16 steps): the recompute reads and writes the state and stores it, the reverse step
    reads the stored state and reads and writes the adjoint; per cell both passes read
    the fields and the reverse step read-modify-writes dL/dE, dL/dB (FP64)."""
    if precision == "fp64":
        packet = 3 * 48 + 3 * 48
        cell = 2 * 48 + 2 * 48
    else:
        packet = 3 * 28 + 28 + 2 * 24         # state read, written, stored, read back; FP32 adjoint read + write
        cell = 2 * 24 + 2 * 48
    return packet + cell / ppc


def algorithmic_bytes_reverse(precision, ppc):
    """Bytes one packet must move at minimum in one reverse-step launch: its stored state
    read and its adjoint (lam_x, lam_u) read and written; per cell, shared by the ppc
    packets, the fields read and dL/dE, dL/dB (FP64) read-modify-written."""
    if precision == "fp64":
        packet = 48 + 2 * 48
        cell = 48 + 2 * 48
    else:
        packet = 28 + 2 * 24                   # cell, offset, u; FP32 adjoint
        cell = 24 + 2 * 48
    return packet + cell / ppc


def copy_bandwidth(nbytes=1 << 31, reps=5):
    """Achieved bandwidth of a plain device-to-device copy (torch copy_) of nbytes, in GB/s
    counting the bytes read and written; median of reps timed copies."""
    import torch
    src = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    times = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        dst.copy_(src)
        b.record()
        torch.cuda.synchronize()
        times.append(a.elapsed_time(b) / 1e3)
    del src, dst
    torch.cuda.empty_cache()
    times.sort()
    return 2 * nbytes / times[len(times) // 2] / 1e9


def measured_traffic(precision, workload, kind="step"):
    """HBM bytes per launch of the step kernel (kind "step") or of the reverse-step kernel
    (kind "reverse") from the committed rocprofv3 counter runs, if they were taken on
    the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
    except Exception:
        return None
    key = f"{workload}:{precision}" + ("" if kind == "step" else f":{kind}")
    rec = data.get(key)
    sources = KERNEL_SOURCES if kind == "step" else REVERSE_SOURCES
    if not rec or rec.get("kernel_hash") != kernel_hash(sources):
        return None
    return rec.get("bytes_per_launch")


def time_path(w, precision, steps, warmup, sort_every, coupled=False, flags=0, losses=False):
    """Time `steps` steps in one call.  coupled=True runs them coupled to the workload's
    seeded gas (rsol_step_coupled: the exchange goes into the gas momentum and energy and
    E is rebuilt from the gas velocity after every step); losses=True adds catastrophic
    losses with the seeded nucleon density and a 4-cell mean free path; flags are
    RSOL_FLAG_* bits."""
    import torch
    from paper_2111_14704_amd.sim import Simulation
    from paper_2111_14704_amd.rsol import RSOL_FLAG_LOSSES
    from workloads import gas_state, loss_state

    sim = Simulation.from_workload(w, precision=precision, sort_every=sort_every,
                                   flags=flags | (RSOL_FLAG_LOSSES if losses else 0))
    h = sim.handle
    if losses:
        nn, sigma, wt = loss_state(w)
        sim.set_losses(10.0 * sigma, nn, wt)
    if coupled:
        rho, mom, egas = (torch.as_tensor(a, dtype=torch.float64, device=sim.device) for a in gas_state(w))

        def run(n):
            sim.step_coupled(n, rho, mom, egas)
    else:
        dM = sim.zeros_grid(3)
        dE = sim.zeros_grid(1)[0]

        def run(n):
            sim.step(n, dM, dE)
    run(warmup)
    h.rsol_check()
    h.rsol_timing(True)
    h.rsol_timing_read()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    step_ms, n_step, sort_ms, n_sort = h.rsol_timing_read()
    h.rsol_timing(False)
    h.rsol_check()
    wall = t1 - t0
    npk = sim.n_particles
    kern_s = step_ms / max(n_step, 1) / 1e3
    balg = algorithmic_bytes_per_packet_step(precision, w.ppc)
    achieved = balg * npk / kern_s / 1e9
    traffic = measured_traffic(precision, w.name.rsplit("-", 1)[0])
    out = dict(
        value=npk * steps / wall, ms_per_step=wall / steps * 1e3,
        kernel_ms=kern_s * 1e3, rebin_ms=(sort_ms / n_sort) if n_sort else 0.0, rebins=n_sort,
        roofline=dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                      traffic=traffic, bytes_per_packet_step=balg, kernel="cells_step_kernel"),
    )
    del sim
    torch.cuda.synchronize()
    return out


def time_one_step_calls(w, precision, calls=20):
    """Wall time of one rsol_step call of one step (the way a code coupled to an MHD
    solver steps), with the packets filed into the cell lists and copied back by every
    call, and with them resident in the lists between calls (RSOL_FLAG_RESIDENT)."""
    import torch
    from paper_2111_14704_amd.rsol import RSOL_FLAG_RESIDENT
    from paper_2111_14704_amd.sim import Simulation
    out = {}
    for name, flags in (("filed_ms", 0), ("resident_ms", RSOL_FLAG_RESIDENT)):
        sim = Simulation.from_workload(w, precision=precision, flags=flags)
        dM, dE = sim.zeros_grid(3), sim.zeros_grid(1)[0]
        for _ in range(3):
            sim.step(1, dM, dE)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(calls):
            sim.step(1, dM, dE)
        torch.cuda.synchronize()
        out[name] = (time.perf_counter() - t0) / calls * 1e3
        sim.sync()
        sim.handle.rsol_check()
        del sim
        torch.cuda.empty_cache()
    return out


def time_backward(precision, nsteps=256, ckpt=16):
    """Differentiation form on workload 5 (32^3 x 32 ppc, CIC): after an untimed two-segment
    warm-up, the forward with checkpoints, then the timed backward (moment adjoint + per
    segment: restore, recompute with stored states, reverse sweep).
    Rate = packets * steps / backward time."""
    import torch
    from paper_2111_14704_amd.autograd import RSOLRollout, spec_from_workload
    from paper_2111_14704_amd.sim import Simulation
    from workloads import make_workload

    w = make_workload(5)
    dev = "cuda"
    # E = -(u/c) x B and the Courant timestep from the library
    sim = Simulation.from_workload(w, precision="fp64")
    dt = sim.dt
    E = sim.E.clone().requires_grad_(True)
    B = sim.B.clone().requires_grad_(True)
    del sim
    x0 = torch.tensor(w.x, device=dev)
    u0 = torch.tensor(w.u, device=dev, requires_grad=True)
    T = torch.tensor(w.target.reshape(3, -1), device=dev)
    spec = spec_from_workload(w, dt, precision)
    # untimed warm-up pass: the first call allocates the handle's scratch and the state
    # slab (through torch's caching allocator, reused by the timed pass)
    rho, P, e = RSOLRollout.apply(E, B, x0, u0, spec, 2 * ckpt, ckpt)
    torch.sqrt(((P - T) ** 2).sum()).backward()
    E.grad = B.grad = u0.grad = None
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rho, P, e = RSOLRollout.apply(E, B, x0, u0, spec, nsteps, ckpt)
    L = torch.sqrt(((P - T) ** 2).sum())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    npk = w.n_particles
    value = npk * nsteps / (t2 - t1)
    balg = algorithmic_bytes_backward(precision, w.ppc)
    achieved = balg * value / 1e9
    # a second, untimed pass with the reverse-step launches bracketed by the library's
    # HIP events (on its stream): the dominant kernel's roofline
    E.grad = B.grad = u0.grad = None
    tspec = dict(spec, time_reverse=True)
    rho, P, e = RSOLRollout.apply(E, B, x0, u0, tspec, nsteps, ckpt)
    torch.sqrt(((P - T) ** 2).sum()).backward()
    torch.cuda.synchronize()
    rev_s = tspec["reverse_ms"] / max(tspec["reverse_launches"], 1) / 1e3
    brev = algorithmic_bytes_reverse(precision, w.ppc)
    rev_launch = brev * npk
    rev_achieved = rev_launch / rev_s / 1e9
    return dict(workload=w.name, dtype="f64" if precision == "fp64" else "f32", value=value,
                unit="particle-updates/s", backward_s=t2 - t1, forward_s=t1 - t0, steps=nsteps, ckpt=ckpt,
                reverse_kernel_us=rev_s * 1e6,
                roofline=dict(bound="hbm", achieved=rev_achieved, peak=HBM_PEAK_GBS, unit="GB/s",
                              frac=rev_achieved / HBM_PEAK_GBS,
                              traffic=measured_traffic(precision, w.name, "reverse"),
                              bytes_per_launch=rev_launch, bytes_per_packet=brev, kernel="step_backward_tiled_kernel",
                              whole_pass=dict(achieved=achieved, frac=achieved / HBM_PEAK_GBS,
                                              bytes_per_packet_step=balg)))


def cpu_baseline(w, sample=1 << 20, steps=10):
    """The CPU oracle (numpy FP64, as it stands) on a bounded sample of the same workload:
    the first `sample` packets for `steps` steps in the workload's fields."""
    import numpy as np
    import oracle
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    p = oracle.Params(w.nx, w.ny, w.nz, w.dx, w.shape, w.c, w.c_tilde, w.qomc,
                      oracle.courant_dt(w.u, w.B, w.c, w.c_tilde, w.qomc, w.dx, w.courant), w.mass)
    E = oracle.electric_field(w.u_gas, w.B, w.c).reshape(3, -1)
    B = w.B.reshape(3, -1)
    x, u = np.ascontiguousarray(w.x[:, :sample]), np.ascontiguousarray(w.u[:, :sample])
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    if ctx:
        ctx.__enter__()
    try:
        t0 = time.perf_counter()
        oracle.rollout(x, u, E, B, p, steps)
        t1 = time.perf_counter()
    finally:
        if ctx:
            ctx.__exit__(None, None, None)
    return dict(value=sample * steps / (t1 - t0), unit="particle-updates/s", cores=1, kind="oracle",
                sample=f"first {sample} packets of the workload, {steps} steps, numpy float64, 1 thread")


def pct_of_peak(value, balg):
    """The metric's "% of HBM peak" on the whole step rate: algorithmic bytes per
    packet-step times packet-steps per second (wall clock over the timed steps, which
    includes the filing of the cell lists, the kernel that adds the exchange into the
    grid and the copy back) against the 8 TB/s peak."""
    return balg * value / 1e9 / HBM_PEAK_GBS


def path_summary(r, precision, w):
    """Fields of one timed path for the JSON line."""
    balg = algorithmic_bytes_per_packet_step(precision, w.ppc)
    return dict(value=r["value"], ms_per_step=r["ms_per_step"], kernel_ms=r["kernel_ms"], rebin_ms=r["rebin_ms"],
                dtype="f64" if precision == "fp64" else "f32", roofline=r["roofline"],
                hbm_frac_full_step=pct_of_peak(r["value"], balg))


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", type=int, default=4, choices=[2, 4],
                    help="headline workload: 4 = 128^3 x 32 ppc turbulence, FP64 and FP32 side by side (default); "
                         "2 = 64^3 x 64 ppc Alfven-mode field")
    ap.add_argument("--extras-workload", type=int, default=2, choices=[2, 4],
                    help="workload of the extra legs (coupled, naive, losses, pushers, one step per call) and of "
                         "the second FP64/FP32 pair")
    ap.add_argument("--no-extras", action="store_true", help="skip every leg on the extras workload")
    ap.add_argument("--sort-every", type=int, default=4, help="re-sort interval of the tiled path (RSOL_FLAG_TILED only)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-backward", action="store_true")
    ap.add_argument("--no-coupled", action="store_true", help="skip the run coupled to the gas")
    ap.add_argument("--no-naive", action="store_true", help="skip the naive-substitution contrast run")
    ap.add_argument("--no-losses", action="store_true", help="skip the run with catastrophic losses")
    ap.add_argument("--no-pushers", action="store_true", help="skip the Vay and Higuera-Cary pusher runs")
    ap.add_argument("--no-one-step", action="store_true", help="skip the one-step-per-call timings")
    ap.add_argument("--no-copy-bw", action="store_true",
                    help="skip the device-copy bandwidth measurement (counter runs keep --calibrate-copy the only copy)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="first run one plain device copy of BYTES bytes (a known-size reference for HBM counters)")
    ap.add_argument("--cpu-sample", type=int, default=1 << 20, help="packets in the CPU oracle's sample")
    ap.add_argument("--cpu-steps", type=int, default=10, help="steps of the CPU oracle's sample")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print(f"bench.py runs on exactly one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding of this path is a design note, not a built feature)", file=sys.stderr)
        sys.exit(2)

    import torch
    from workloads import make_workload

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.calibrate_copy:
        n = args.calibrate_copy // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy of {n * 8} bytes done", file=sys.stderr, flush=True)
        del src, dst
    w = make_workload(args.workload, precision="fp64")
    base = w.name.rsplit("-", 1)[0]
    print(f"[bench] workload {base}: {w.n_particles} packets, {w.nx}^3 cells", file=sys.stderr, flush=True)
    r64 = time_path(w, "fp64", args.steps, args.warmup, args.sort_every)
    print(f"[bench] fp64 {r64['value']:.3e} upd/s, kernel {r64['kernel_ms']:.3f} ms", file=sys.stderr, flush=True)
    r32 = None
    if not args.no_fp32:
        r32 = time_path(w, "fp32", args.steps, args.warmup, args.sort_every)
        print(f"[bench] fp32 {r32['value']:.3e} upd/s, kernel {r32['kernel_ms']:.3f} ms", file=sys.stderr, flush=True)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(w, sample=args.cpu_sample, steps=args.cpu_steps)
        print(f"[bench] cpu oracle {cpu['value']:.3e} upd/s", file=sys.stderr, flush=True)
    cfg = dict(workload=base, grid=[w.nx, w.ny, w.nz], ppc=w.ppc, n_particles=w.n_particles, shape=w.shape,
               c_over_c_tilde=w.c / w.c_tilde, steps_per_call=args.steps, parallelism="none")
    del w

    extras = {}
    if not args.no_extras:
        w2 = make_workload(args.extras_workload, precision="fp64")
        b2 = w2.name.rsplit("-", 1)[0]
        ex = dict(workload=b2, n_particles=w2.n_particles)
        print(f"[bench] extras on {b2}: {w2.n_particles} packets", file=sys.stderr, flush=True)
        if args.extras_workload != args.workload:
            e64 = time_path(w2, "fp64", args.steps, args.warmup, args.sort_every)
            ex["fp64"] = path_summary(e64, "fp64", w2)
            print(f"[bench] {b2} fp64 {e64['value']:.3e} upd/s, kernel {e64['kernel_ms']:.3f} ms", file=sys.stderr,
                  flush=True)
            if not args.no_fp32:
                e32 = time_path(w2, "fp32", args.steps, args.warmup, args.sort_every)
                ex["fp32"] = path_summary(e32, "fp32", w2)
                ex["fp32"]["speedup_vs_fp64"] = e32["value"] / e64["value"]
                print(f"[bench] {b2} fp32 {e32['value']:.3e} upd/s, kernel {e32['kernel_ms']:.3f} ms",
                      file=sys.stderr, flush=True)
            ref_ms = e64["ms_per_step"]
        else:
            ref_ms = r64["ms_per_step"]
        if not args.no_coupled:
            rc = time_path(w2, "fp64", args.steps, args.warmup, args.sort_every, coupled=True)
            ex["coupled"] = dict(value=rc["value"], ms_per_step=rc["ms_per_step"], kernel_ms=rc["kernel_ms"],
                                 dtype="f64", overhead_vs_static=rc["ms_per_step"] / ref_ms - 1.0)
            print(f"[bench] coupled fp64 {rc['value']:.3e} upd/s, kernel {rc['kernel_ms']:.3f} ms", file=sys.stderr,
                  flush=True)
        if not args.no_naive:
            from paper_2111_14704_amd.rsol import RSOL_FLAG_NAIVE
            rn = time_path(w2, "fp64", args.steps, args.warmup, args.sort_every, flags=RSOL_FLAG_NAIVE)
            ex["naive"] = dict(value=rn["value"], ms_per_step=rn["ms_per_step"], kernel_ms=rn["kernel_ms"],
                               dtype="f64")
            print(f"[bench] naive fp64 {rn['value']:.3e} upd/s, kernel {rn['kernel_ms']:.3f} ms", file=sys.stderr,
                  flush=True)
        if not args.no_losses:
            rl = time_path(w2, "fp64", args.steps, args.warmup, args.sort_every, losses=True)
            ex["losses"] = dict(value=rl["value"], ms_per_step=rl["ms_per_step"], kernel_ms=rl["kernel_ms"],
                                dtype="f64", overhead_vs_static=rl["ms_per_step"] / ref_ms - 1.0)
            print(f"[bench] losses fp64 {rl['value']:.3e} upd/s, kernel {rl['kernel_ms']:.3f} ms", file=sys.stderr,
                  flush=True)
        if not args.no_pushers:
            from paper_2111_14704_amd.rsol import RSOL_FLAG_PUSHER_HC, RSOL_FLAG_PUSHER_VAY
            rp = {}
            for name, fl in (("vay", RSOL_FLAG_PUSHER_VAY), ("hc", RSOL_FLAG_PUSHER_HC)):
                r = time_path(w2, "fp64", args.steps, args.warmup, args.sort_every, flags=fl)
                rp[name] = dict(value=r["value"], ms_per_step=r["ms_per_step"], kernel_ms=r["kernel_ms"], dtype="f64")
                print(f"[bench] {name} pusher fp64 {r['value']:.3e} upd/s, kernel {r['kernel_ms']:.3f} ms",
                      file=sys.stderr, flush=True)
            ex["pushers"] = rp
        if not args.no_one_step:
            one = {}
            for prec in ("fp64", "fp32"):
                one[prec] = time_one_step_calls(w2, prec)
                print(f"[bench] one step per call {prec}: {one[prec]['filed_ms']:.3f} ms filed, "
                      f"{one[prec]['resident_ms']:.3f} ms resident", file=sys.stderr, flush=True)
            ex["one_step_calls"] = one
        del w2
        extras = ex
    bwd = None
    if not args.no_backward:
        bwd = time_backward("fp64")
        print(f"[bench] backward fp64 {bwd['value']:.3e} upd/s, reverse kernel {bwd['reverse_kernel_us']:.1f} us",
              file=sys.stderr, flush=True)
        b32 = time_backward("fp32")
        bwd["fp32"] = dict(value=b32["value"], backward_s=b32["backward_s"], reverse_kernel_us=b32["reverse_kernel_us"],
                           roofline=b32["roofline"],
                           reverse_time_vs_fp64=b32["reverse_kernel_us"] / bwd["reverse_kernel_us"])
        print(f"[bench] backward fp32 {b32['value']:.3e} upd/s, reverse kernel {b32['reverse_kernel_us']:.1f} us",
              file=sys.stderr, flush=True)
    if not args.no_copy_bw:
        copy_gbs = copy_bandwidth()
        print(f"[bench] device copy {copy_gbs:.0f} GB/s", file=sys.stderr, flush=True)
        rooflines = [r64["roofline"], r32 and r32["roofline"], bwd and bwd["roofline"],
                     bwd and bwd["fp32"]["roofline"]]
        for k in ("fp64", "fp32"):
            if k in extras:
                rooflines.append(extras[k]["roofline"])
        for rf in rooflines:
            if rf:
                rf["copy_gbs"] = copy_gbs
                rf["frac_of_copy"] = rf["achieved"] / copy_gbs

    balg64 = algorithmic_bytes_per_packet_step("fp64", cfg["ppc"])
    line = dict(
        metric=METRIC, value=r64["value"], unit="particle-updates/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=r64["ms_per_step"], higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f64", data="synthetic",
        config=cfg,
        roofline=r64["roofline"],
        hbm_frac_full_step=pct_of_peak(r64["value"], balg64),
        cpu_baseline=cpu,
        kernel_ms=r64["kernel_ms"], rebin_ms=r64["rebin_ms"],
    )
    if r32:
        line["fp32"] = dict(path_summary(r32, "fp32", _Cfg(cfg["ppc"])), speedup_vs_fp64=r32["value"] / r64["value"],
                            kernel_speedup_vs_fp64=r64["kernel_ms"] / r32["kernel_ms"])
    if extras:
        line["extras"] = extras
    if bwd:
        line["backward"] = bwd
    print(json.dumps(line), flush=True)


class _Cfg:
    """The one workload attribute path_summary needs once the workload itself is freed."""

    def __init__(self, ppc):
        self.ppc = ppc


if __name__ == "__main__":
    main()
