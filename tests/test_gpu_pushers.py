"""Parity of the alternative pushers (RSOL_FLAG_PUSHER_VAY, RSOL_FLAG_PUSHER_HC) with the
oracle's Vay and Higuera-Cary updates, through the C ABI: the cell-list and keep-order
steps, the separate push phase, combined with losses, and at full size on a sample.

Tolerances as in the Boris parity tests: FP64 1e-10, FP32 1e-5."""

import math
import sys

import numpy as np
import pytest

import oracle
from workloads import make_workload, loss_state
from tests.helpers import oracle_params, oracle_fields, periodic_distance, rel_l2, rel_linf, max_rel_momentum

pytestmark = pytest.mark.gpu

KEEP_ORDER, TILED, LOSSES, VAY, HC = 1, 2, 8, 16, 32
PUSHERS = {"vay": VAY, "hc": HC}


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _params(w, dt, pusher):
    return oracle.Params(w.nx, w.ny, w.nz, w.dx, w.shape, w.c, w.c_tilde, w.qomc, dt, w.mass, pusher=pusher)


def _check(w, nsteps, pusher, flags, tol, label):
    import torch
    from paper_2111_14704_amd.sim import Simulation
    sim = Simulation.from_workload(w, flags=flags | PUSHERS[pusher])
    dM, dE = sim.zeros_grid(3), sim.zeros_grid(1)[0]
    sim.step(nsteps, dM, dE)
    sim.handle.rsol_check()
    torch.cuda.synchronize()
    x, u = sim.state_by_id()
    E, B = oracle_fields(w)
    p = _params(w, sim.dt, pusher)
    r = oracle.rollout(w.x, w.u, E, B, p, nsteps)
    dist = float(np.max(periodic_distance(x, r["x"], w.box)))
    g = np.sqrt(1 + np.sum(w.u ** 2, axis=0)).mean()
    escale = (p.c / p.c_tilde) * p.mass * p.c ** 2 * g * w.ppc * math.sqrt(w.n_cells) / p.volume
    errs = dict(x_cells=dist / w.dx, u=max_rel_momentum(u, r["u"]), dM=rel_l2(dM.cpu().numpy(), r["dM_sum"]), dM_inf=rel_linf(dM.cpu().numpy(), r["dM_sum"]),
                dE_abs=float(np.linalg.norm(dE.cpu().numpy() - r["dE_sum"]) / escale))
    _say(f"{label}: " + ", ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= tol, (label, k, v)


@pytest.mark.parametrize("pusher", ["vay", "hc"])
@pytest.mark.parametrize("flags", [0, KEEP_ORDER], ids=["cells", "global"])
def test_pusher_config1_fp64(pusher, flags):
    """Workload 1 (16^3, 8 ppc, CIC), 40 steps."""
    w = make_workload(1)
    _say(f"{pusher} config1 flags={flags}")
    _check(w, 40, pusher, flags, 1e-10, f"{pusher} config1 flags={flags}")


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
@pytest.mark.parametrize("pusher", ["vay", "hc"])
@pytest.mark.parametrize("flags", [0, KEEP_ORDER], ids=["cells", "global"])
def test_pusher_alfven_ragged(precision, tol, pusher, flags):
    """Workload 2 recipe on a ragged 10^3 grid (TSC, 4 ppc), 20 steps."""
    w = make_workload(2, n=10, ppc=4, precision=precision)
    _say(f"{pusher} alfven n=10 {precision} flags={flags}")
    _check(w, 20, pusher, flags, tol, f"{pusher} alfven {precision} flags={flags}")


@pytest.mark.parametrize("pusher", ["vay", "hc"])
def test_pusher_keeps_the_force_free_drift(pusher):
    """Packets on a lattice in the force-free E x B state of a uniform flow across B: the
    Vay and Higuera-Cary updates leave their momenta unchanged (to rounding) for 200 steps,
    and they drift at (c_tilde/c) u_gas."""
    import torch
    from paper_2111_14704_amd.sim import Simulation
    n, U = 8, 1.0
    w = make_workload(1, n=n, ppc=1)
    nc = n ** 3
    i = np.arange(nc)
    w.x = np.stack([i % n, i // n % n, i // (n * n)]).astype(float) + 0.5
    beta = U / w.c
    w.u = np.tile(np.array([[0.0], [beta / math.sqrt(1 - beta ** 2)], [0.0]]), (1, nc))
    w.ids = np.arange(nc, dtype=np.int32)
    w.u_gas = np.zeros((3, n, n, n))
    w.u_gas[1] = U
    _say(f"{pusher} force-free drift")
    sim = Simulation.from_workload(w, flags=PUSHERS[pusher], dt=0.3 / w.c_tilde)
    sim.step(200)
    sim.handle.rsol_check()
    torch.cuda.synchronize()
    x, u = sim.state_by_id()
    assert np.max(np.abs(u - w.u)) <= 1e-13 * w.u[1, 0]
    shift = (x[1] - w.x[1]) % n
    assert np.max(np.abs(shift - (w.c_tilde / w.c) * U * 200 * sim.dt)) < 1e-9


@pytest.mark.parametrize("pusher", ["vay", "hc"])
def test_pusher_separate_phases(pusher):
    """rsol_gather, rsol_push (with the pusher), rsol_deposit and rsol_drift reproduce one
    oracle step."""
    import torch
    from paper_2111_14704_amd.sim import Simulation
    w = make_workload(2, n=8, ppc=4)
    _say(f"{pusher} separate phases")
    sim = Simulation.from_workload(w, flags=KEEP_ORDER | PUSHERS[pusher])
    h = sim.handle
    f64 = dict(dtype=torch.float64, device=sim.device)
    Ep, Bp = torch.empty((3, w.n_particles), **f64), torch.empty((3, w.n_particles), **f64)
    pay = torch.empty((4, w.n_particles), **f64)
    dM, dE = sim.zeros_grid(3), sim.zeros_grid(1)[0]
    h.rsol_gather(Ep, Bp)
    h.rsol_push(Ep, Bp, pay)
    h.rsol_deposit(pay, dM, dE)
    h.rsol_drift()
    h.rsol_check()
    torch.cuda.synchronize()
    x, u = sim.state_by_id()
    E, B = oracle_fields(w)
    x1, u1, dM1, dE1 = oracle.step(w.x, w.u, E, B, _params(w, sim.dt, pusher))
    assert np.max(periodic_distance(x, x1, w.box)) <= 1e-12
    assert max_rel_momentum(u, u1) <= 1e-12
    assert rel_l2(dM.cpu().numpy(), dM1) <= 1e-10


def test_pusher_with_losses():
    """Higuera-Cary with catastrophic losses on the cell-list path, 20 steps."""
    import torch
    from paper_2111_14704_amd.sim import Simulation
    w = make_workload(2, n=10, ppc=4)
    nn, sigma, wt = loss_state(w)
    _say("hc with losses")
    sim = Simulation.from_workload(w, flags=LOSSES | HC)
    sim.set_losses(10 * sigma, nn, wt)
    dM = sim.zeros_grid(3)
    sim.step(20, dM, None)
    sim.handle.rsol_check()
    torch.cuda.synchronize()
    x, u = sim.state_by_id()
    E, B = oracle_fields(w)
    r = oracle.rollout_with_losses(w.x, w.u, wt, E, B, nn, 10 * sigma, _params(w, sim.dt, "hc"), 20)
    assert float(np.max(periodic_distance(x, r["x"], w.box))) / w.dx <= 1e-10
    assert max_rel_momentum(u, r["u"]) <= 1e-10
    assert float(np.max(np.abs(sim.weights_by_id() - r["w"]) / r["w"])) <= 1e-10
    assert rel_l2(dM.cpu().numpy(), r["dM_sum"]) <= 1e-10


@pytest.mark.parametrize("pusher", ["vay", "hc"])
def test_pusher_full_size_sampled(pusher):
    """Full-size workload 2 (16.8M packets) on the cell-list path, 30 steps; 2048 packets
    sampled by id re-run one by one in the oracle."""
    import torch
    from paper_2111_14704_amd.sim import Simulation
    w = make_workload(2)
    nsteps = 30
    _say(f"{pusher} full-size workload 2, {w.n_particles} packets")
    sim = Simulation.from_workload(w, flags=PUSHERS[pusher])
    sim.step(nsteps)
    sim.handle.rsol_check()
    torch.cuda.synchronize()
    pick = np.sort(np.random.default_rng(77).choice(w.n_particles, 2048, replace=False))
    ids = sim.ids.cpu().numpy()
    where = np.empty(w.n_particles, dtype=np.int64)
    where[ids] = np.arange(w.n_particles)
    sel = torch.as_tensor(where[pick], device=sim.device)
    xg = sim.positions64()[:, sel].cpu().numpy()
    ug = sim.u[:, sel].double().cpu().numpy()
    E, B = oracle_fields(w)
    r = oracle.rollout(w.x[:, pick], w.u[:, pick], E, B, _params(w, sim.dt, pusher), nsteps)
    dist = float(np.max(periodic_distance(xg, r["x"], w.box)))
    eu = max_rel_momentum(ug, r["u"])
    _say(f"{pusher} full size: x_cells={dist:.2e} e_u={eu:.2e}")
    assert dist / w.dx <= 1e-10 and eu <= 1e-10


def test_pusher_flags_rejected_where_not_served():
    """Both pusher flags, the tiled path with a non-Boris pusher and the differentiation
    form with one are refused with RSOL_EINVAL."""
    import torch
    from paper_2111_14704_amd.rsol import RSOLError
    from paper_2111_14704_amd.sim import Simulation
    w = make_workload(1, n=8, ppc=1)
    _say("pusher rejections")
    for flags in (VAY | HC, TILED | VAY):
        with pytest.raises(RSOLError) as ei:
            Simulation.from_workload(w, flags=flags)
        assert ei.value.code == -1
    sim = Simulation.from_workload(w, flags=VAY)
    with pytest.raises(RSOLError) as ei:
        sim.handle.rsol_set_flags(VAY | TILED)
    assert ei.value.code == -1
    states = torch.empty(sim.handle.rsol_state_bytes(), dtype=torch.uint8, device=sim.device)
    with pytest.raises(RSOLError) as ei:
        sim.handle.rsol_record_states(1, states)
    assert ei.value.code == -1
