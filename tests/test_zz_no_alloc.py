"""rsol_step_static, the allocation-free variant of rsol_step (scratch in a static device
array of the library), against rsol_step on a handle with caller scratch: two calls in a
row on the same GPU, the second with fewer packets, then an FP32 call; the same packets
and the same exchange to the parity bar (1e-10 FP64, the FP32 form's rounding in FP32).
Also: a problem larger than the static array is refused with RSOL_ESCRATCH."""

import sys

import numpy as np
import pytest

from workloads import make_workload
from tests.helpers import periodic_distance, rel_l2, rel_linf, max_rel_momentum

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _static_run(w, sim_ref, nsteps):
    """The same steps through rsol_step_static on fresh copies of the workload's packets."""
    import torch
    from paper_2111_14704_amd import rsol
    dev = "cuda"
    p = rsol.Params(**{k: getattr(sim_ref.params, k) for k in ("nx", "ny", "nz", "shape", "precision", "dx", "c",
                                                                "c_tilde", "qomc", "courant", "mass", "sort_every",
                                                                "flags")})
    p.dt = sim_ref.dt
    ids = torch.as_tensor(w.ids, device=dev)
    x64 = torch.as_tensor(np.ascontiguousarray(w.x), dtype=torch.float64, device=dev)
    if w.precision == "fp32":
        # the handle's own conversion gives the same cell + offset the reference used
        cell = torch.empty(w.n_particles, dtype=torch.int32, device=dev)
        off = torch.empty((3, w.n_particles), dtype=torch.float32, device=dev)
        sim_ref.handle.rsol_positions_to_cells(x64, cell, off)
        u = torch.as_tensor(np.ascontiguousarray(w.u), dtype=torch.float32, device=dev)
        pos = cell
    else:
        pos, off = x64, None
        u = torch.as_tensor(np.ascontiguousarray(w.u), dtype=torch.float64, device=dev)
    dM = torch.zeros((3, w.n_cells), dtype=torch.float64, device=dev)
    dE = torch.zeros(w.n_cells, dtype=torch.float64, device=dev)
    rsol.rsol_step_static(p, pos, off, u, ids, sim_ref.E, sim_ref.B, nsteps, dM, dE)
    torch.cuda.synchronize()
    if w.precision == "fp32":
        x = torch.empty((3, w.n_particles), dtype=torch.float64, device=dev)
        sim_ref.handle.rsol_cells_to_positions(pos, off, x)
    else:
        x = pos
    order = np.argsort(ids.cpu().numpy(), kind="stable")
    return (x.cpu().numpy()[:, order], u.double().cpu().numpy()[:, order], dM.cpu().numpy(), dE.cpu().numpy())


def _reference(w, nsteps):
    import torch
    from paper_2111_14704_amd.sim import Simulation
    sim = Simulation.from_workload(w)
    dM, dE = sim.zeros_grid(3), sim.zeros_grid(1)[0]
    sim.step(nsteps, dM, dE)
    sim.handle.rsol_check()
    torch.cuda.synchronize()
    x, u = sim.state_by_id()
    return sim, x, u, dM.cpu().numpy(), dE.cpu().numpy()


@pytest.mark.parametrize("calls", [[(1, 16, 8, "fp64"), (2, 8, 4, "fp64"), (3, 12, 2, "fp32")]])
def test_static_scratch_step_matches_rsol_step(calls):
    for k, n, ppc, precision in calls:
        w = make_workload(k, n=n, ppc=ppc, precision=precision)
        _say(f"rsol_step_static workload {k} n={n} ppc={ppc} {precision} np={w.n_particles}")
        sim, xr, ur, dMr, dEr = _reference(w, 10)
        xs, us, dMs, dEs = _static_run(w, sim, 10)
        fp64 = precision == "fp64"
        ex = float(np.max(periodic_distance(xs, xr, w.box))) / w.dx
        eu = max_rel_momentum(us, ur)
        em, emi = rel_l2(dMs, dMr), rel_linf(dMs, dMr)
        # the energy exchange is a small difference of packet energies (zero in real
        # arithmetic in workload 1's pure B): compare against its natural per-cell scale
        g = float(np.sqrt(1 + np.sum(w.u ** 2, axis=0)).mean())
        scale = (w.c / w.c_tilde) * w.mass * w.c ** 2 * g * ppc / w.dx ** 3
        ee = float(np.max(np.abs(dEs - dEr))) / scale
        _say(f"  x_cells={ex:.2e} u={eu:.2e} dM={em:.2e} dM_inf={emi:.2e} dE_inf={ee:.2e}")
        tol = 1e-10 if fp64 else 1e-5
        assert ex <= tol and eu <= tol and em <= tol and emi <= tol and ee <= tol


def test_static_scratch_refuses_a_problem_too_large():
    import torch
    from paper_2111_14704_amd import rsol
    p = rsol.Params(nx=64, ny=64, nz=64, shape=rsol.RSOL_TSC, precision=rsol.RSOL_FP64, dx=1.0, c=1000.0,
                    c_tilde=100.0, qomc=4000.0, dt=1e-3)
    npk = 1 << 20
    assert rsol.rsol_scratch_bytes(p, npk) > (64 << 20)
    dev = "cuda"
    x = torch.zeros((3, npk), dtype=torch.float64, device=dev)
    u = torch.zeros_like(x)
    ids = torch.zeros(npk, dtype=torch.int32, device=dev)
    E = torch.zeros((3, 64 ** 3), dtype=torch.float64, device=dev)
    with pytest.raises(rsol.RSOLError) as ei:
        rsol.rsol_step_static(p, x, None, u, ids, E, E, 1)
    assert ei.value.code == -6
    assert "static scratch" in str(ei.value)
