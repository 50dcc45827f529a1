"""Reference gradients of the momentum-density loss, for checking the
hand-written adjoint.  TEST INFRASTRUCTURE ONLY (see the package docstring).

Loss: L = || P_N - T ||_2 with P_N the CR momentum density (Sec. 2, packet
totals P_j = M_j c u_j spread by W) after N packet steps from (x^0, u^{-1/2})
in static grid fields, and T a fixed target.  The timestep is a fixed
hyper-parameter, not differentiated.

Two independent estimators of dL/dtheta for a single coordinate theta (a
grid E or B component in one cell, or one packet's initial momentum
component):
  * complex step (Squire & Trapp 1998): Im L(theta + i h) / h with h = 1e-30,
    exact to rounding with no subtractive cancellation;
  * central difference with step h, evaluated so that the unperturbed part
    of the sum cancels exactly.
Both are "structured": with static fields packets do not interact, so only
the packets whose trajectory can feel theta are re-run and the rest of P_N
enters as a fixed sum.  This is the chain rule dL/dtheta = sum_i dL/dP_i dP_i/dtheta
with dL/dP_i = (P_i - T_i)/L, applied exactly.
"""

from __future__ import annotations

import math

import numpy as np

from .pic import Params, moments, shape_weights, step


def momentum_loss(P, T):
    """L = sqrt(sum (P - T)^2), written without abs() so it stays analytic."""
    d = (P - T).ravel()
    return np.sqrt(np.sum(d * d))


def final_momentum_density(x0, u0, E, B, p: Params, nsteps):
    x, u = x0, u0
    for _ in range(nsteps):
        x, u, _, _ = step(x, u, E, B, p)
    _, P, _ = moments(x, u, p)
    return P


def packets_touching(x0, u0, E, B, p: Params, nsteps, cells):
    """For each cell in ``cells``, the packets whose gather stencil contains it
    at some step 0..nsteps-1 (those are the only packets that feel a change of
    E or B in that cell)."""
    cells = np.asarray(sorted(set(int(c) for c in cells)))
    hit = {int(c): set() for c in cells}
    x, u = x0, u0
    for _ in range(nsteps):
        idx, _ = shape_weights(x, p)
        mask = np.isin(idx, cells)
        rows, cols = np.nonzero(mask)
        for r, cc in zip(rows, idx[rows, cols]):
            hit[int(cc)].add(int(r))
        x, u, _, _ = step(x, u, E, B, p)
    return {c: np.array(sorted(s), dtype=np.int64) for c, s in hit.items()}


def _perturbed_inputs(kind, comp, where, E, B, u0, sub, delta):
    """Inputs of the packet subset ``sub`` with theta moved by ``delta``."""
    Ep, Bp, up = E, B, u0[:, sub]
    if kind == "E":
        Ep = E.astype(np.result_type(E, delta)).copy()
        Ep[comp, where] += delta
    elif kind == "B":
        Bp = B.astype(np.result_type(B, delta)).copy()
        Bp[comp, where] += delta
    elif kind == "u":
        up = up.astype(np.result_type(up, delta)).copy()
        j = int(np.nonzero(sub == where)[0][0])
        up[comp, j] += delta
    else:
        raise ValueError(kind)
    return Ep, Bp, up


def _subset(kind, where, touching):
    if kind == "u":
        return np.array([where], dtype=np.int64)
    return touching[where]


def complex_step_grad(x0, u0, E, B, p: Params, nsteps, T, coords, touching=None, h=1e-30):
    """dL/dtheta for each (kind, comp, where) in ``coords`` by complex step."""
    P0 = final_momentum_density(x0, u0, E, B, p, nsteps)
    L0 = float(np.real(momentum_loss(P0, T)))
    gL = (P0 - T) / L0
    out = []
    for kind, comp, where in coords:
        sub = _subset(kind, where, touching)
        if sub.size == 0:
            out.append(0.0)
            continue
        Ep, Bp, up = _perturbed_inputs(kind, comp, where, E, B, u0, sub, 1j * h)
        Psub = final_momentum_density(x0[:, sub].astype(complex), up.astype(complex), Ep, Bp, p, nsteps)
        out.append(float(np.sum(gL * (np.imag(Psub) / h))))
    return np.array(out), L0


def central_fd_grad(x0, u0, E, B, p: Params, nsteps, T, coords, touching=None, h=1e-6):
    """dL/dtheta by central differences (L(theta+h) - L(theta-h)) / 2h, with the
    unperturbed packets' contribution cancelled exactly and exact summation."""
    P0 = final_momentum_density(x0, u0, E, B, p, nsteps)
    out = []
    for kind, comp, where in coords:
        sub = _subset(kind, where, touching)
        if sub.size == 0:
            out.append(0.0)
            continue
        Pbase = final_momentum_density(x0[:, sub], u0[:, sub], E, B, p, nsteps)
        rest = P0 - Pbase
        vals = []
        for sgn in (1.0, -1.0):
            Ep, Bp, up = _perturbed_inputs(kind, comp, where, E, B, u0, sub, sgn * h)
            Ps = final_momentum_density(x0[:, sub], up, Ep, Bp, p, nsteps)
            vals.append(Ps)
        # L+^2 - L-^2 = sum (P+ - P-)(P+ + P- - 2T), with P+ - P- touching only the subset
        diff = (vals[0] - vals[1]).ravel()
        summ = (2.0 * rest + vals[0] + vals[1] - 2.0 * T).ravel()
        l2p = math.fsum(((rest + vals[0] - T) ** 2).ravel())
        l2m = math.fsum(((rest + vals[1] - T) ** 2).ravel())
        dl2 = math.fsum(diff * summ)
        out.append(dl2 / (math.sqrt(l2p) + math.sqrt(l2m)) / (2.0 * h))
    return np.array(out)
