"""Parity of the naive-substitution contrast mode (RSOL_FLAG_NAIVE) with the oracle's
naive mode, through the C ABI: the same kernels with the naive constants (electric and
magnetic half kicks (c/c_tilde) q dt/(2 m c) and q dt/(2 m c), packet momentum and
energy with c_tilde, no c/c_tilde on the back-reaction).

Tolerances as in the RSOL parity tests: FP64 1e-10, FP32 1e-5 (positions relative to
the box and in cells, momenta per packet, exchange and moments relative L2).  The
energy exchange is compared absolutely against the naive per-cell packet energy scale
M c_tilde^2 gamma."""

import math
import sys

import numpy as np
import pytest

import oracle
from workloads import make_workload, gas_state
from tests.helpers import oracle_fields, periodic_distance, rel_l2, rel_linf, max_rel_momentum

pytestmark = pytest.mark.gpu

NAIVE = 4


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _naive_params(w, dt):
    return oracle.Params(w.nx, w.ny, w.nz, w.dx, w.shape, w.c, w.c_tilde, w.qomc, dt, w.mass, naive=True)


def _gpu(w, nsteps, flags):
    import torch
    from paper_2111_14704_amd.sim import Simulation
    sim = Simulation.from_workload(w, flags=flags | NAIVE)
    dM, dE = sim.zeros_grid(3), sim.zeros_grid(1)[0]
    sim.step(nsteps, dM, dE)
    sim.handle.rsol_check()
    rho, P, e = sim.moments()
    torch.cuda.synchronize()
    x, u = sim.state_by_id()
    return dict(x=x, u=u, dM=dM.cpu().numpy(), dE=dE.cpu().numpy(), rho=rho.cpu().numpy(), P=P.cpu().numpy(),
                e=e.cpu().numpy(), dt=sim.dt)


def _oracle(w, nsteps, dt):
    p = _naive_params(w, dt)
    E, B = oracle_fields(w)
    r = oracle.rollout(w.x, w.u, E, B, p, nsteps)
    r["rho"], r["P"], r["e"] = oracle.moments(r["x"], r["u"], p)
    r["p"] = p
    return r


def _compare(w, got, ref, tol, label):
    p = ref["p"]
    dist = float(np.max(periodic_distance(got["x"], ref["x"], w.box)))
    g = np.sqrt(1 + np.sum(w.u ** 2, axis=0)).mean()
    escale = p.mass * p.c_tilde ** 2 * g * w.ppc * math.sqrt(w.n_cells) / p.volume
    errs = dict(x_cells=dist / w.dx, u=max_rel_momentum(got["u"], ref["u"]), dM=rel_l2(got["dM_sum"], ref["dM_sum"]), dM_inf=rel_linf(got["dM_sum"], ref["dM_sum"]),
                dE_abs=float(np.linalg.norm(got["dE"] - ref["dE_sum"]) / escale),
                rho=rel_l2(got["rho"], ref["rho"]), rho_inf=rel_linf(got["rho"], ref["rho"]), P=rel_l2(got["P"], ref["P"]), P_inf=rel_linf(got["P"], ref["P"]), e=rel_l2(got["e"], ref["e"]), e_inf=rel_linf(got["e"], ref["e"]))
    _say(f"{label}: " + ", ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= tol, (label, k, v)


def _check(w, nsteps, flags, tol, label):
    got = _gpu(w, nsteps, flags)
    got["dM_sum"] = got["dM"]
    ref = _oracle(w, nsteps, got["dt"])
    _compare(w, got, ref, tol, label)


@pytest.mark.parametrize("flags", [0, 2, 1], ids=["cells", "tiled", "global"])
def test_naive_config1_fp64(flags):
    """Workload 1 (16^3, 8 ppc, CIC, c/c_tilde = 10), 40 naive steps."""
    w = make_workload(1)
    _say(f"naive config1 fp64 flags={flags}")
    _check(w, 40, flags, 1e-10, f"naive config1 flags={flags}")


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
@pytest.mark.parametrize("flags", [0, 2, 1], ids=["cells", "tiled", "global"])
def test_naive_alfven_ragged(precision, tol, flags):
    """Workload 2 recipe on a ragged 10^3 grid, TSC, 4 ppc, 20 naive steps."""
    w = make_workload(2, n=10, ppc=4, precision=precision)
    _say(f"naive alfven n=10 {precision} flags={flags}")
    _check(w, 20, flags, tol, f"naive alfven {precision} flags={flags}")


def test_naive_courant_dt_matches_oracle():
    """The naive gyro limit uses the unreduced q|B|/(gamma m c)."""
    from paper_2111_14704_amd.sim import Simulation
    for k in (1, 2):
        w = make_workload(k, n=16, ppc=4)
        _say(f"naive dt workload {k}")
        sim = Simulation.from_workload(w, flags=NAIVE)
        want = oracle.courant_dt(w.u, w.B, w.c, w.c_tilde, w.qomc, w.dx, w.courant, naive=True)
        assert sim.dt == pytest.approx(want, rel=1e-15)


def test_naive_coupled_to_the_gas():
    """The naive mode coupled to the gas (rsol_step_coupled): its own momentum and energy
    totals (M c_tilde u, M c_tilde^2 gamma, no c/c_tilde) are the ones kept."""
    import torch
    from paper_2111_14704_amd.sim import Simulation
    w = make_workload(2, n=10, ppc=4)
    rho, mom, egas = gas_state(w)
    _say("naive coupled")
    sim = Simulation.from_workload(w, flags=NAIVE)
    f64 = dict(dtype=torch.float64, device=sim.device)
    t_rho, t_mom, t_eg = (torch.as_tensor(a, **f64) for a in (rho, mom, egas))
    sim.step_coupled(20, t_rho, t_mom, t_eg)
    sim.handle.rsol_check()
    torch.cuda.synchronize()
    x, u = sim.state_by_id()
    p = _naive_params(w, sim.dt)
    r = oracle.coupled_rollout(w.x, w.u, mom, egas, rho, w.B.reshape(3, -1), p, 20)
    assert float(np.max(periodic_distance(x, r["x"], w.box))) / w.dx <= 1e-10
    assert max_rel_momentum(u, r["u"]) <= 1e-10
    assert rel_l2(t_mom.cpu().numpy() - mom, r["mom"] - mom) <= 1e-10
    assert rel_l2(sim.E.cpu().numpy(), r["E"]) <= 1e-10
    P0, E0 = oracle.conserved_totals(w.u, mom, egas, p)
    P1, E1 = oracle.conserved_totals(u, t_mom.cpu().numpy(), t_eg.cpu().numpy(), p)
    scale = p.mass * p.c_tilde * np.abs(w.u).sum() + np.abs(mom).sum()
    assert np.all(np.abs(P1 - P0) <= 1e-12 * scale)


def test_naive_full_size_sampled():
    """Workload 2 at full size (16.8M packets) in the naive mode on the cell-list path,
    30 steps; 2048 packets sampled by id re-run one by one in the oracle."""
    import torch
    from paper_2111_14704_amd.sim import Simulation
    w = make_workload(2)
    nsteps = 30
    _say(f"naive full-size workload 2, {w.n_particles} packets")
    sim = Simulation.from_workload(w, flags=NAIVE)
    dM = sim.zeros_grid(3)
    sim.step(nsteps, dM, None)
    sim.handle.rsol_check()
    torch.cuda.synchronize()
    pick = np.sort(np.random.default_rng(321).choice(w.n_particles, 2048, replace=False))
    ids = sim.ids.cpu().numpy()
    where = np.empty(w.n_particles, dtype=np.int64)
    where[ids] = np.arange(w.n_particles)
    sel = torch.as_tensor(where[pick], device=sim.device)
    xg = sim.positions64()[:, sel].cpu().numpy()
    ug = sim.u[:, sel].double().cpu().numpy()
    E, B = oracle_fields(w)
    r = oracle.rollout(w.x[:, pick], w.u[:, pick], E, B, _naive_params(w, sim.dt), nsteps)
    dist = float(np.max(periodic_distance(xg, r["x"], w.box)))
    eu = max_rel_momentum(ug, r["u"])
    _say(f"naive full size: x_cells={dist:.2e} e_u={eu:.2e}")
    assert dist / w.dx <= 1e-10 and eu <= 1e-10


def test_naive_is_rejected_by_the_differentiation_form():
    import torch
    from paper_2111_14704_amd.rsol import RSOLError
    from paper_2111_14704_amd.sim import Simulation
    w = make_workload(1, n=8, ppc=1)
    _say("naive adjoint rejected")
    sim = Simulation.from_workload(w, flags=NAIVE)
    states = torch.empty(sim.handle.rsol_state_bytes(), dtype=torch.uint8, device=sim.device)
    with pytest.raises(RSOLError) as ei:
        sim.handle.rsol_record_states(1, states)
    assert ei.value.code == -1
