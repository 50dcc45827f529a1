"""Test-side glue: oracle parameters from a workload, error metrics."""

from __future__ import annotations

import numpy as np

import oracle


def oracle_params(w, dt=None):
    """oracle.Params for workload ``w``; dt from the oracle's timestep rule unless given."""
    if dt is None:
        dt = oracle.courant_dt(w.u, w.B, w.c, w.c_tilde, w.qomc, w.dx, w.courant)
    return oracle.Params(w.nx, w.ny, w.nz, w.dx, w.shape, w.c, w.c_tilde, w.qomc, dt, w.mass)


def oracle_fields(w):
    """(E, B) as (3, n_cells) arrays, E from the oracle's E = -(u/c) x B."""
    E = oracle.electric_field(w.u_gas, w.B, w.c).reshape(3, -1)
    return E, w.B.reshape(3, -1)


def periodic_distance(a, b, box):
    """Per-packet minimum-image distance between two (3, Np) position arrays."""
    d = np.abs(a - b)
    for k in range(3):
        d[k] = np.minimum(d[k], box[k] - d[k])
    return np.sqrt(np.sum(d * d, axis=0))


def rel_l2(a, ref):
    a = np.asarray(a, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    den = np.linalg.norm(ref)
    return float(np.linalg.norm(a - ref) / (den if den > 0 else 1.0))


def max_rel_momentum(u, ref):
    """max_j |u_j - u_j^ref| / |u_j^ref|."""
    return float(np.max(np.linalg.norm(u - ref, axis=0) / np.linalg.norm(ref, axis=0)))


def rel_linf(a, ref):
    """max |a - ref| over every cell and component, relative to max |ref|: one cell far
    off fails it where the grid-wide relative L2 would dilute it."""
    a = np.asarray(a, dtype=np.float64).ravel()
    ref = np.asarray(ref, dtype=np.float64).ravel()
    den = np.max(np.abs(ref)) if ref.size else 0.0
    return float(np.max(np.abs(a - ref)) / (den if den > 0 else 1.0)) if a.size else 0.0


def round_to_fp32_state(x, u, dx):
    """The packet state as the precision form stores it: home cell = floor(x/dx) plus an
    in-cell offset rounded to float32 (an offset that rounds up to 1 becomes 0 of the next
    cell), and the momentum rounded to float32.  Returned as float64 arrays again."""
    s = np.asarray(x, dtype=np.float64) / dx
    c = np.floor(s)
    f = (s - c).astype(np.float32).astype(np.float64)
    up = f >= 1.0
    f = np.where(up, 0.0, f)
    c = np.where(up, c + 1.0, c)
    return (c + f) * dx, np.asarray(u, dtype=np.float32).astype(np.float64)


def fp32_storage_rollout(x, u, E, B, p, nsteps):
    """The oracle's steps (FP64 arithmetic) with the packet state rounded to the precision
    form's storage before the first step and after every step.  Against the plain oracle
    this gives the error that storing the state in the FP32 form costs by itself,
    whatever the arithmetic; returns the oracle rollout's dict keys x, u, dM, dE,
    dM_sum, dE_sum."""
    box = np.array([p.nx * p.dx, p.ny * p.dx, p.nz * p.dx])[:, None]
    x, u = round_to_fp32_state(x, u, p.dx)
    x = np.where(x >= box, x - box, x)
    dM_sum = np.zeros((3, p.n_cells))
    dE_sum = np.zeros(p.n_cells)
    dM = dE = None
    for _ in range(nsteps):
        x, u, dM, dE = oracle.step(x, u, E, B, p)
        dM_sum = dM_sum + dM
        dE_sum = dE_sum + dE
        x, u = round_to_fp32_state(x, u, p.dx)
        x = np.where(x >= box, x - box, x)
    return dict(x=x, u=u, dM=dM, dE=dE, dM_sum=dM_sum, dE_sum=dE_sum)
