"""Write tests/golden/workload5_gradients.json: the CPU oracle's gradients of the
workload-5 loss L = || P_N - T ||_2 (CR momentum density after 256 steps, 32^3 grid,
32 packets per cell, CIC) at the workload's 64 sampled coordinates (16 of E, 16 of B,
32 of the initial momenta).

Two estimators, both from oracle/ only:
  * complex step, h = 1e-30 (exact to rounding);
  * central difference, h = 1e-6, with the unperturbed packets' part of P cancelled
    exactly and exact (fsum) summation; a coordinate whose +-h runs move any affected
    packet across a CIC kink (a change of the lower node index at any step) is marked
    rejected, since the loss is only piecewise smooth there.
Only the packets a coordinate can affect are re-run (fields are static, so packets do
not interact): one packet for a momentum coordinate, the packets whose stencil ever
contains the cell for a field coordinate.

Usage: python tests/golden/make_workload5_gradients.py [--procs 8]
"""

import argparse
import json
import math
import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import adjoint  # noqa: E402
from oracle.pic import shape_weights, step, moments  # noqa: E402
from workloads import make_workload  # noqa: E402

W = None
P = None
E = None
B = None
NSTEPS = 256


def _setup():
    global W, P, E, B
    W = make_workload(5)
    dt = oracle.courant_dt(W.u, W.B, W.c, W.c_tilde, W.qomc, W.dx, W.courant)
    P = oracle.Params(W.nx, W.ny, W.nz, W.dx, W.shape, W.c, W.c_tilde, W.qomc, dt, W.mass)
    E = oracle.electric_field(W.u_gas, W.B, W.c).reshape(3, -1)
    B = W.B.reshape(3, -1)


def _base_chunk(args):
    """Final momentum density of a packet chunk and, for the target cells, which packets
    of the chunk have the cell in their stencil at some step."""
    lo, hi, cells = args
    if W is None:
        _setup()
    x, u = W.x[:, lo:hi], W.u[:, lo:hi]
    cells = np.asarray(cells)
    hit = {int(c): set() for c in cells}
    for _ in range(NSTEPS):
        idx, _ = shape_weights(x, P)
        rows, cols = np.nonzero(np.isin(idx, cells))
        for r, cc in zip(rows, idx[rows, cols]):
            hit[int(cc)].add(lo + int(r))
        x, u, _, _ = step(x, u, E, B, P)
    _, Pm, _ = moments(x, u, P)
    return Pm, {c: sorted(s) for c, s in hit.items()}


def _run_subset(x0, u0, Ec, Bc):
    """Final momentum density of a packet subset and the lower CIC node index at every step."""
    x, u = x0, u0
    trace = []
    for _ in range(NSTEPS):
        trace.append(np.floor(np.real(x) / P.dx - 0.5).astype(np.int64))
        x, u, _, _ = step(x, u, Ec, Bc, P)
    _, Pm, _ = moments(x, u, P)
    return Pm, np.array(trace)


def _coord(args):
    kind, comp, where, sub, gL_list, P0_list, T_list = args
    if W is None:
        _setup()
    sub = np.asarray(sub, dtype=np.int64)
    gL, P0, T = np.asarray(gL_list), np.asarray(P0_list), np.asarray(T_list)
    if sub.size == 0:
        return dict(cs=0.0, fd=0.0, rejected=False, n=0)
    x0, u0 = W.x[:, sub], W.u[:, sub]

    def inputs(delta):
        Ec, Bc, uc = E, B, u0
        if kind == "E":
            Ec = E.astype(np.result_type(E, delta)).copy()
            Ec[comp, where] += delta
        elif kind == "B":
            Bc = B.astype(np.result_type(B, delta)).copy()
            Bc[comp, where] += delta
        else:
            uc = u0.astype(np.result_type(u0, delta)).copy()
            uc[comp, int(np.nonzero(sub == where)[0][0])] += delta
        return Ec, Bc, uc

    # complex step
    Ec, Bc, uc = inputs(1e-30j)
    Pc, _ = _run_subset(x0.astype(complex), uc.astype(complex), Ec, Bc)
    cs = float(np.sum(gL * np.imag(Pc) / 1e-30))
    # central difference with exact cancellation of the untouched packets
    Pb, tb = _run_subset(x0, u0, E, B)
    rest = P0 - Pb
    outs, rejected = [], False
    for sgn in (1.0, -1.0):
        Ec, Bc, uc = inputs(sgn * 1e-6)
        Ps, ts = _run_subset(x0, uc, Ec, Bc)
        rejected |= bool(np.any(ts != tb))
        outs.append(Ps)
    diff = (outs[0] - outs[1]).ravel()
    summ = (2.0 * rest + outs[0] + outs[1] - 2.0 * T).ravel()
    l2p = math.fsum(((rest + outs[0] - T) ** 2).ravel())
    l2m = math.fsum(((rest + outs[1] - T) ** 2).ravel())
    fd = math.fsum(diff * summ) / (math.sqrt(l2p) + math.sqrt(l2m)) / 2e-6
    return dict(cs=cs, fd=fd, rejected=rejected, n=int(sub.size))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=8)
    ap.add_argument("--out", default=os.path.join(HERE, "workload5_gradients.json"))
    args = ap.parse_args()
    _setup()
    coords = W.grad_coords
    cells = sorted({c for k, _, c in coords if k != "u"})
    npk = W.n_particles
    chunks = np.linspace(0, npk, 4 * args.procs + 1).astype(int)
    with mp.Pool(args.procs) as pool:
        parts = pool.map(_base_chunk, [(int(a), int(b), cells) for a, b in zip(chunks[:-1], chunks[1:])])
        P0 = sum(pm for pm, _ in parts)
        touch = {c: sorted(set().union(*[set(h[c]) for _, h in parts])) for c in cells}
        T = W.target.reshape(3, -1)
        L0 = float(np.sqrt(np.sum((P0 - T) ** 2)))
        gL = (P0 - T) / L0
        jobs = []
        for kind, comp, where in coords:
            sub = [where] if kind == "u" else touch[where]
            jobs.append((kind, comp, where, sub, gL, P0, T))
        res = pool.map(_coord, jobs, chunksize=1)
    out = dict(
        workload=W.name, nsteps=NSTEPS, dt=P.dt, loss=L0,
        coords=[[k, c, i] for k, c, i in coords],
        complex_step=[r["cs"] for r in res], central_difference=[r["fd"] for r in res],
        fd_rejected=[r["rejected"] for r in res], packets_rerun=[r["n"] for r in res],
        note="oracle gradients of L = ||P_N - T||_2; dt is the oracle's Courant timestep, held fixed",
    )
    with open(args.out, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {args.out}: L = {L0:.6e}, rejected FD {sum(out['fd_rejected'])} of {len(coords)}")


if __name__ == "__main__":
    main()
