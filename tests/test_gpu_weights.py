"""Per-packet weights on the default path (rsol_set_weights, no losses): a packet stands
for N_j particles (Sec. 2, Eq. (4); Sec. 4 sets N_j from the total mass or energy), so
its mass M_j = mass * w_j scales its exchange (Eq. (12)) and its moments.  Compared with
the oracle's weighted step (step_with_losses at zero cross-section) through the C ABI on
the cell-list path (one call, and one step per call with resident lists) and the
keep-order path: packets, weights (unchanged), summed exchange and weighted moments,
FP64 at 1e-10 and FP32 at 1e-5.  Paths that carry no weights refuse them."""

import sys

import numpy as np
import pytest

import oracle
from workloads import make_workload
from tests.helpers import oracle_params, oracle_fields, periodic_distance, rel_l2, rel_linf, max_rel_momentum

pytestmark = pytest.mark.gpu

WEIGHTS, KEEP_ORDER, TILED, RESIDENT = 8, 1, 2, 64


def _say(msg):
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def _weights(w):
    return np.random.default_rng(21).uniform(0.2, 2.0, w.n_particles)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-10), ("fp32", 1e-5)])
@pytest.mark.parametrize("flags,per_call", [(0, 20), (RESIDENT, 1), (KEEP_ORDER, 20)],
                         ids=["cells", "resident-1-per-call", "keep-order"])
def test_weighted_packets_match_oracle(precision, tol, flags, per_call):
    import torch
    from paper_2111_14704_amd.sim import Simulation
    w = make_workload(2, n=16, ppc=8, nsteps=20, precision=precision)
    wt = _weights(w)
    _say(f"weights {precision} flags={flags} per_call={per_call}")
    sim = Simulation.from_workload(w, flags=flags | WEIGHTS)
    sim.set_weights(wt)
    dM, dE = sim.zeros_grid(3), sim.zeros_grid(1)[0]
    done = 0
    while done < 20:
        n = min(per_call, 20 - done)
        sim.step(n, dM, dE)
        done += n
    sim.handle.rsol_check()
    rho, P, e = sim.moments()
    torch.cuda.synchronize()
    x, u = sim.state_by_id()
    gw = sim.weights_by_id()
    p = oracle_params(w)
    assert abs(sim.dt - p.dt) <= (1e-6 if precision == "fp32" else 1e-14) * p.dt
    p.dt = sim.dt
    E, B = oracle_fields(w)
    r = oracle.rollout_with_losses(w.x, w.u, wt, E, B, np.zeros(w.n_cells), 0.0, p, 20)
    rr, rP, re = oracle.moments(r["x"], r["u"], p, w=r["w"])
    g = float(np.sqrt(1 + np.sum(w.u ** 2, axis=0)).mean())
    escale = (p.c / p.c_tilde) * p.mass * p.c ** 2 * g * w.ppc * np.sqrt(w.n_cells) / p.volume
    errs = dict(x_cells=float(np.max(periodic_distance(x, r["x"], w.box))) / w.dx, u=max_rel_momentum(u, r["u"]),
                w=float(np.max(np.abs(gw - r["w"]) / r["w"])),
                dM=rel_l2(dM.cpu().numpy(), r["dM_sum"]), dM_inf=rel_linf(dM.cpu().numpy(), r["dM_sum"]),
                dE_abs=float(np.linalg.norm(dE.cpu().numpy() - r["dE_sum"]) / escale),
                rho=rel_l2(rho.cpu().numpy(), rr), rho_inf=rel_linf(rho.cpu().numpy(), rr),
                P=rel_l2(P.cpu().numpy(), rP), P_inf=rel_linf(P.cpu().numpy(), rP),
                e=rel_l2(e.cpu().numpy(), re), e_inf=rel_linf(e.cpu().numpy(), re))
    _say(f"weights {precision} flags={flags}: " + ", ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= tol, (k, v)
    # the weights matter: the unweighted exchange differs
    r1 = oracle.rollout(w.x, w.u, E, B, p, 20)
    assert rel_l2(r1["dM_sum"], r["dM_sum"]) > 1e-2


def test_paths_without_weights_refuse_them():
    import torch
    from paper_2111_14704_amd.rsol import RSOLError
    from paper_2111_14704_amd.sim import Simulation
    w = make_workload(2, n=8, ppc=2)
    _say("weights refused by the tiled path, the separate phases and the sort")
    sim = Simulation.from_workload(w, flags=WEIGHTS | TILED)
    with pytest.raises(RSOLError) as ei:
        sim.set_weights(_weights(w))
    assert ei.value.code == -1
    sim = Simulation.from_workload(w, flags=WEIGHTS)
    sim.set_weights(_weights(w))
    f64 = dict(dtype=torch.float64, device="cuda")
    Ep, Bp = torch.empty((3, w.n_particles), **f64), torch.empty((3, w.n_particles), **f64)
    for call in (lambda: sim.handle.rsol_gather(Ep, Bp), lambda: sim.handle.rsol_sort(),
                 lambda: sim.handle.rsol_set_flags(WEIGHTS | TILED)):
        with pytest.raises(RSOLError) as ei:
            call()
        assert ei.value.code == -1
    sim2 = Simulation.from_workload(w)
    with pytest.raises(RSOLError) as ei:
        sim2.set_weights(_weights(w))
    assert ei.value.code == -2
