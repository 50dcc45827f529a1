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
