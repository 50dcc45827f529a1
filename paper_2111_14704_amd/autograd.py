"""torch.autograd binding of the differentiation form.

``RSOLRollout.apply(E, B, x0, u0, spec, nsteps, ckpt)`` runs ``nsteps`` packet steps
from (x0, u0) in the static grid fields E, B (no exchange deposit) and returns the CR
moments (rho, P, e) of the final state.  Its backward runs the library's hand-written
adjoint: the adjoint of the moment deposit (a gather) at the final state, then, segment
by segment from the last checkpoint back, a recompute that stores every state of the
segment followed by the reverse sweep of the step adjoint (drift, Boris kick, and the
gather, whose adjoint is a scatter into dL/dE and dL/dB).  Checkpoints are taken every
``ckpt`` steps.  dt is a fixed parameter (not differentiated).

Packet order: the packets are re-binned once (rank-major cell order, so neighbouring
lanes sit in different cells) and then kept in that order for the whole rollout so
checkpoints, stored states and adjoint arrays stay aligned; gradients are returned in
the caller's packet order.  (Inside the library the recompute and the reverse sweep
work on copies sorted by tile every four steps; the arrays seen here keep their order.)
"""

from __future__ import annotations

import torch

from .rsol import (RSOL_CIC, RSOL_FLAG_KEEP_ORDER, RSOL_FLAG_RECORD_ONLY, RSOL_FP32, RSOL_FP64, RSOL_TSC, Handle,
                   Params)


def _params(spec):
    return Params(nx=spec["nx"], ny=spec["ny"], nz=spec["nz"], shape=RSOL_CIC if spec["shape"] == "cic" else RSOL_TSC,
                  precision=RSOL_FP32 if spec.get("precision", "fp64") == "fp32" else RSOL_FP64, dx=spec["dx"],
                  c=spec["c"], c_tilde=spec["c_tilde"], qomc=spec["qomc"], dt=spec["dt"],
                  courant=spec.get("courant", 0.3), mass=spec["mass"], sort_every=1, flags=0)


class _Run:
    """Handle plus the packet-state tensors it is registered with."""

    def __init__(self, spec, E, B, x0, u0):
        self.fp32 = spec.get("precision", "fp64") == "fp32"
        dev = E.device
        npk = x0.shape[1]
        self.n = npk
        self.h = Handle(_params(spec), npk, device=dev)
        self.E = E.detach().contiguous()
        self.B = B.detach().contiguous()
        self.h.rsol_set_fields(self.E, self.B)
        self.ids = torch.arange(npk, dtype=torch.int32, device=dev)
        if self.fp32:
            self.cell = torch.empty(npk, dtype=torch.int32, device=dev)
            self.off = torch.empty((3, npk), dtype=torch.float32, device=dev)
            if npk:
                self.h.rsol_positions_to_cells(x0.detach().double().contiguous(), self.cell, self.off)
            self.u = u0.detach().float().contiguous().clone()
            self.state = [self.cell, self.off, self.u]
            self.h.rsol_set_particles(self.cell, self.off, self.u, self.ids)
        else:
            self.x = x0.detach().double().contiguous().clone()
            self.u = u0.detach().double().contiguous().clone()
            self.state = [self.x, self.u]
            self.h.rsol_set_particles(self.x, None, self.u, self.ids)
        self.h.rsol_set_dt(spec["dt"])
        if npk:
            self.h.rsol_sort()
        self.h.rsol_set_flags(RSOL_FLAG_KEEP_ORDER)

    def snapshot(self):
        return [t.clone() for t in self.state]

    def restore(self, snap):
        for dst, src in zip(self.state, snap):
            dst.copy_(src)

    def lam_dtype(self):
        return torch.float32 if self.fp32 else torch.float64


class RSOLRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, E, B, x0, u0, spec, nsteps, ckpt):
        run = _Run(spec, E, B, x0, u0)
        ckpts = []
        done = 0
        while done < nsteps:
            seg = min(ckpt, nsteps - done)
            ckpts.append((run.snapshot(), seg))
            run.h.rsol_step(seg)
            done += seg
        rho = torch.zeros(run.E.shape[1], dtype=torch.float64, device=E.device)
        P = torch.zeros_like(run.E)
        e = torch.zeros_like(rho)
        run.h.rsol_moments(rho, P, e)
        ctx.run = run
        ctx.ckpts = ckpts
        ctx.spec = spec
        return rho, P, e

    @staticmethod
    def backward(ctx, g_rho, g_P, g_e):
        run, ckpts = ctx.run, ctx.ckpts
        h = run.h
        dev = run.E.device
        lam_x = torch.zeros((3, run.n), dtype=run.lam_dtype(), device=dev)
        lam_u = torch.zeros_like(lam_x)
        gE = torch.zeros_like(run.E)
        gB = torch.zeros_like(run.B)
        if run.n:
            c = lambda t: None if t is None else t.detach().double().contiguous()  # noqa: E731
            h.rsol_moments_backward(lam_x, lam_u, lam_rho=c(g_rho), lam_P=c(g_P), lam_e=c(g_e))
            slab = h.rsol_state_bytes()
            longest = max(seg for _, seg in ckpts)
            states = torch.empty(slab * longest, dtype=torch.uint8, device=dev)
            # spec["time_reverse"]: time the reverse-step launches alone with the
            # library's launch events (a profiling aid; it synchronises once per segment)
            # and leave their summed milliseconds and count in the spec
            timing = bool(ctx.spec.get("time_reverse"))
            rev_ms, rev_n = 0.0, 0
            # each segment restores its checkpoint before recording, so the recording
            # need not bring the packets back into the run's arrays
            h.rsol_set_flags(RSOL_FLAG_KEEP_ORDER | RSOL_FLAG_RECORD_ONLY)
            for snap, seg in reversed(ckpts):
                run.restore(snap)
                h.rsol_record_states(seg, states)
                if timing:
                    h.rsol_timing(True)
                h.rsol_step_backward(seg, states, lam_x, lam_u, gE, gB)
                if timing:
                    ms, n, _, _ = h.rsol_timing_read()
                    h.rsol_timing(False)
                    rev_ms += ms
                    rev_n += n
            h.rsol_set_flags(RSOL_FLAG_KEEP_ORDER)
            if timing:
                ctx.spec["reverse_ms"] = rev_ms
                ctx.spec["reverse_launches"] = rev_n
        order = run.ids.long()
        gx = torch.zeros((3, run.n), dtype=torch.float64, device=dev)
        gu = torch.zeros_like(gx)
        gx[:, order] = lam_x.double()
        gu[:, order] = lam_u.double()
        ctx.run = None
        ctx.ckpts = None
        ctx.spec = None
        return gE, gB, gx, gu, None, None, None


def rollout_moments(E, B, x0, u0, spec, nsteps, ckpt=16):
    """(rho, P, e) after nsteps steps; differentiable w.r.t. E, B, x0 and u0."""
    return RSOLRollout.apply(E, B, x0, u0, spec, int(nsteps), int(ckpt))


def spec_from_workload(w, dt, precision=None):
    return dict(nx=w.nx, ny=w.ny, nz=w.nz, dx=w.dx, shape=w.shape, c=w.c, c_tilde=w.c_tilde, qomc=w.qomc,
                courant=w.courant, mass=w.mass, dt=float(dt), precision=precision or w.precision)
