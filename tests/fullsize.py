"""The oracle's step and moments over every packet of a full-size workload, in chunks
spread over worker processes (packets are independent given the fields; only the
deposits are summed).  Test-side glue: the arithmetic is the oracle's."""

from __future__ import annotations

import multiprocessing as mp
import os

import numpy as np

import oracle

_G = {}


def _workers():
    # the GPU machine gives one GPU's share of its cores (16); never more than the host has
    return max(1, min(16, os.cpu_count() or 1))


def _step_part(k):
    x, u, E, B, p, chunks = _G["x"], _G["u"], _G["E"], _G["B"], _G["p"], _G["chunks"]
    dM = np.zeros((3, p.n_cells))
    dE = np.zeros(p.n_cells)
    outs = []
    for c in range(k, len(chunks), _G["nw"]):
        a, b = chunks[c]
        x1, u1, m, e = oracle.step(x[:, a:b], u[:, a:b], E, B, p)
        dM += m
        dE += e
        outs.append((a, b, x1, u1))
    return dM, dE, outs


def _moments_part(k):
    x, u, p, chunks = _G["x"], _G["u"], _G["p"], _G["chunks"]
    acc = [np.zeros(p.n_cells), np.zeros((3, p.n_cells)), np.zeros(p.n_cells)]
    for c in range(k, len(chunks), _G["nw"]):
        a, b = chunks[c]
        r, P, e = oracle.moments(x[:, a:b], u[:, a:b], p)
        acc[0] += r
        acc[1] += P
        acc[2] += e
    return acc


def _run(fn, x, u, p, E=None, B=None, chunk=1 << 20):
    n = x.shape[1]
    chunks = [(a, min(n, a + chunk)) for a in range(0, n, chunk)]
    nw = min(_workers(), len(chunks))
    _G.update(x=x, u=u, E=E, B=B, p=p, chunks=chunks, nw=nw)
    try:
        ctx = mp.get_context("fork")
        with ctx.Pool(nw) as pool:
            return pool.map(fn, range(nw))
    finally:
        _G.clear()


def oracle_step_all(x, u, E, B, p, chunk=1 << 20):
    """oracle.step over every packet: (x1, u1, dM, dE)."""
    parts = _run(_step_part, x, u, p, E, B, chunk)
    x1 = np.empty_like(x)
    u1 = np.empty_like(u)
    dM = np.zeros((3, p.n_cells))
    dE = np.zeros(p.n_cells)
    for m, e, outs in parts:
        dM += m
        dE += e
        for a, b, xa, ua in outs:
            x1[:, a:b] = xa
            u1[:, a:b] = ua
    return x1, u1, dM, dE


def oracle_moments_all(x, u, p, chunk=1 << 20):
    """oracle.moments over every packet: (rho, P, e)."""
    parts = _run(_moments_part, x, u, p, chunk=chunk)
    rho = sum(q[0] for q in parts)
    P = sum(q[1] for q in parts)
    e = sum(q[2] for q in parts)
    return rho, P, e
