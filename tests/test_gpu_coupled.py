"""Parity of the coupled step (rsol_step_coupled: packets plus a gas whose density and
magnetic field are held fixed) with the oracle's coupled rollout, through the C ABI.

Every step gathers E = -(u_gas/c) x B with u_gas = mom/rho, the gas takes the step's
exchange (Eq. (12)) and E is rebuilt before the next step, so the packets feel the gas
they push.  Compared: packet positions and momenta by id (as in the static-field
parity tests), the gas momentum gained over the run (relative L2), the gas energy
gained (absolute, against the per-cell packet energy scale (c/c_tilde) M c^2 gamma),
and the final E (relative L2).  Tolerances: FP64 path 1e-10, FP32 precision form 1e-5.
At full size the oracle cannot follow every packet, so the run is checked through what
holds at any size: the conserved momentum and energy totals (Sec. 2, discussion after
Eq. (12)) and E of the final gas state."""

import math
import sys

import numpy as np
import pytest

import oracle
from workloads import make_workload, gas_state
from tests.helpers import oracle_params, periodic_distance, rel_l2, rel_linf, max_rel_momentum

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _gpu_coupled(w, nsteps, gas, per_call=None, **kw):
    import torch
    from paper_2111_14704_amd.sim import Simulation
    sim = Simulation.from_workload(w, **kw)
    f64 = dict(dtype=torch.float64, device=sim.device)
    rho, mom, egas = (torch.as_tensor(np.ascontiguousarray(a), **f64) for a in gas)
    per_call = per_call or max(nsteps, 1)
    done = 0
    while True:
        n = min(per_call, nsteps - done)
        sim.step_coupled(n, rho, mom, egas)
        done += n
        if done >= nsteps:
            break
    sim.handle.rsol_check()
    torch.cuda.synchronize()
    x, u = sim.state_by_id()
    return dict(x=x, u=u, mom=mom.cpu().numpy(), egas=egas.cpu().numpy(), E=sim.E.cpu().numpy(), dt=sim.dt)


def _oracle_coupled(w, nsteps, gas, dt):
    p = oracle_params(w, dt=dt)
    rho, mom, egas = gas
    r = oracle.coupled_rollout(w.x, w.u, mom, egas, rho, w.B.reshape(3, -1), p, nsteps)
    r["p"] = p
    return r


def _energy_scale(w, p):
    g = np.sqrt(1 + np.sum(w.u ** 2, axis=0)).mean()
    return (p.c / p.c_tilde) * p.mass * p.c ** 2 * g * max(w.n_particles / w.n_cells, 1.0) * math.sqrt(w.n_cells) / p.volume


def _compare(w, gas, got, ref, tol, label):
    p = ref["p"]
    _, mom0, egas0 = gas
    dist = float(np.max(periodic_distance(got["x"], ref["x"], w.box))) if w.n_particles else 0.0
    errs = dict(x_cells=dist / w.dx,
                u=max_rel_momentum(got["u"], ref["u"]) if w.n_particles else 0.0,
                mom=rel_l2(got["mom"] - mom0, ref["mom"] - mom0), mom_inf=rel_linf(got["mom"] - mom0, ref["mom"] - mom0),
                egas_abs=float(np.linalg.norm(got["egas"] - ref["egas"]) / _energy_scale(w, p)),
                E=rel_l2(got["E"], ref["E"]), E_inf=rel_linf(got["E"], ref["E"]))
    _say(f"{label}: " + ", ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= tol, (label, k, v)


@pytest.mark.parametrize("flags", [0, 2, 1], ids=["cells", "tiled", "global"])
def test_coupled_config1_fp64(flags):
    """Workload 1 (16^3, 8 ppc, CIC, c/c_tilde = 10), 20 coupled steps in one call."""
    w = make_workload(1)
    gas = gas_state(w)
    _say(f"coupled config1 fp64 flags={flags}")
    got = _gpu_coupled(w, 20, gas, flags=flags)
    _compare(w, gas, got, _oracle_coupled(w, 20, gas, got["dt"]), 1e-10, f"coupled config1 flags={flags}")


@pytest.mark.parametrize("flags", [0, 2], ids=["cells", "tiled"])
def test_coupled_config3_fp32(flags):
    """Workload 3 (the FP32 precision form of workload 1), 20 coupled steps."""
    w = make_workload(3)
    gas = gas_state(w)
    _say(f"coupled config3 fp32 flags={flags}")
    got = _gpu_coupled(w, 20, gas, flags=flags)
    _compare(w, gas, got, _oracle_coupled(w, 20, gas, got["dt"]), 1e-5, f"coupled config3 flags={flags}")


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
@pytest.mark.parametrize("flags,per_call", [(0, 20), (0, 3), (2, 20), (1, 20), (64, 1), (64, 3)],
                         ids=["cells", "cells-3-per-call", "tiled", "global", "resident-1-per-call",
                              "resident-3-per-call"])
def test_coupled_alfven_ragged(precision, tol, flags, per_call):
    """Workload 2 recipe on a 10^3 grid (ragged 4^3 tiles), TSC, 4 ppc, 20 steps: the gas
    flow of the Alfven modes changes by tens of percent, enough to move the packets well
    above the tolerances, so a stale or wrong E fails."""
    w = make_workload(2, n=10, ppc=4, precision=precision)
    gas = gas_state(w)
    _say(f"coupled alfven n=10 {precision} flags={flags} per_call={per_call}")
    got = _gpu_coupled(w, 20, gas, per_call=per_call, flags=flags)
    _compare(w, gas, got, _oracle_coupled(w, 20, gas, got["dt"]), tol,
             f"coupled alfven {precision} flags={flags} per_call={per_call}")


def _lattice(n, precision):
    """One packet per cell on the cell centres, all with u = (0, 1, 0) across B = x_hat, and
    a uniform gas of density 2 holding minus (c/c_tilde) times the CR momentum: the
    zero-momentum frame of the oracle's closed-form coupled gyration."""
    w = make_workload(1, n=n, ppc=1, precision=precision)
    nc = n ** 3
    i = np.arange(nc)
    w.x = np.stack([i % n, i // n % n, i // (n * n)]).astype(float) + 0.5
    w.u = np.tile(np.array([0.0, 1.0, 0.0])[:, None], (1, nc))
    w.ids = np.arange(nc, dtype=np.int32)
    w.mass = 0.14
    w.c_tilde = 100.0
    w.B = np.zeros((3, n, n, n))
    w.B[0] = 1.0
    w.u_gas = np.zeros((3, n, n, n))
    rho = np.full(nc, 2.0)
    mom = np.tile((-(w.c / w.c_tilde) * w.mass * w.c * w.u[:, :1]), (1, nc))
    return w, (rho, np.ascontiguousarray(mom), np.zeros(nc))


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
@pytest.mark.parametrize("flags", [0, 2, 1], ids=["cells", "tiled", "global"])
def test_coupled_lattice_gyration(precision, tol, flags):
    """The strongly coupled closed-form case (gas term as large as the packet term of the
    gyration rate), 100 steps of dt = 2.5e-5 (about a third of a turn)."""
    w, gas = _lattice(4, precision)
    _say(f"coupled lattice {precision} flags={flags}")
    got = _gpu_coupled(w, 100, gas, dt=2.5e-5, flags=flags)
    _compare(w, gas, got, _oracle_coupled(w, 100, gas, got["dt"]), tol, f"lattice {precision} flags={flags}")


def test_coupled_no_packets_and_zero_steps():
    """Without packets, or with nsteps = 0, the gas is unchanged and E is the field of
    the given gas momentum."""
    import torch
    from paper_2111_14704_amd.sim import Simulation
    w = make_workload(2, n=8, ppc=2)
    rho, mom, egas = gas_state(w)
    E_ref = oracle.electric_field(mom / rho, w.B.reshape(3, -1), w.c)
    _say("coupled empty / zero steps")
    for case in ("empty", "zero-steps"):
        kw = dict(x=np.zeros((3, 0)), u=np.zeros((3, 0)), ids=np.zeros(0, np.int32), dt=1e-3) \
            if case == "empty" else {}
        sim = Simulation.from_workload(w, **kw)
        sim.E.zero_()
        f64 = dict(dtype=torch.float64, device=sim.device)
        t_rho, t_mom, t_eg = (torch.as_tensor(a, **f64) for a in (rho, mom, egas))
        sim.step_coupled(3 if case == "empty" else 0, t_rho, t_mom, t_eg)
        sim.handle.rsol_check()
        torch.cuda.synchronize()
        assert np.array_equal(t_mom.cpu().numpy(), mom) and np.array_equal(t_eg.cpu().numpy(), egas), case
        assert rel_l2(sim.E.cpu().numpy(), E_ref) <= 1e-14, case


def test_coupled_full_size_config2_conservation():
    """Workload 2 at full size (64^3 x 64 ppc, 16.8M packets, TSC, FP64), 10 coupled
    steps on the cell-list path: V sum mom + (c/c_tilde) M c sum u and V sum egas +
    (c/c_tilde) M c^2 sum gamma are unchanged up to rounding, and E is the field of the
    final gas momentum."""
    import torch
    w = make_workload(2)
    gas = gas_state(w)
    rho, mom0, egas0 = gas
    _say(f"coupled full-size config2, {w.n_particles} packets")
    got = _gpu_coupled(w, 10, gas)
    p = oracle_params(w, dt=got["dt"])
    k = p.c / p.c_tilde
    P0, En0 = oracle.conserved_totals(w.u, mom0, egas0, p)
    P1, En1 = oracle.conserved_totals(got["u"], got["mom"], got["egas"], p)
    # rounding of the per-cell sums of each step's deposit and of these totals
    scale_p = k * p.mass * p.c * np.abs(w.u).sum() + p.volume * np.abs(mom0).sum()
    scale_e = k * p.mass * p.c ** 2 * oracle.lorentz_gamma(w.u).sum() + p.volume * egas0.sum()
    res_p = np.abs(P1 - P0) / scale_p
    res_e = abs(En1 - En0) / scale_e
    _say(f"momentum residual {res_p}, energy residual {res_e:.2e}, mom change "
         f"{rel_l2(got['mom'], mom0):.2e}")
    assert np.all(res_p <= 1e-12) and res_e <= 1e-12
    assert rel_l2(got["mom"], mom0) > 1e-3          # the gas did take up momentum
    E_ref = oracle.electric_field(got["mom"] / rho, w.B.reshape(3, -1), w.c)
    assert rel_l2(got["E"], E_ref) <= 1e-14
