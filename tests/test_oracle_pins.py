"""Pins of the CPU oracle against what the paper and the mathematics fix,
independent of the oracle's own formulas: closed forms of the gyro motion and
the E x B drift, invariants, the c_tilde-scaling laws of the RSOL
formulation, textbook assignment weights, a high-order ODE solve of the
continuous equations, and brute-force cross checks."""

from fractions import Fraction
import math
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from oracle import adjoint
from workloads import make_workload, loss_state
from tests.helpers import oracle_params, oracle_fields

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _uniform_params(n, shape, ratio, dt=None, c=1000.0, qomc=4000.0, mass=1.0):
    return oracle.Params(n, n, n, 1.0, shape, c, c / ratio, qomc, dt if dt is not None else 0.0, mass)


def _uniform_fields(n, B=(1.0, 0.0, 0.0), u_gas=(0.0, 0.0, 0.0), c=1000.0):
    nc = n ** 3
    Bg = np.tile(np.asarray(B, float)[:, None], (1, nc))
    ug = np.tile(np.asarray(u_gas, float)[:, None], (1, nc))
    return oracle.electric_field(ug, Bg, c), Bg


# ---------------------------------------------------------------- spatial kernel W

def test_shape_weights_golden():
    """Hand-worked CIC/TSC weights (tests/golden/shape_weights.txt, Hockney & Eastwood
    Sec. 5-3), the kernel W of the packet decomposition, Sec. 2 Eq. (4).  The packet sits at
    (s, s, s) so the 3-D weight of node (a, b, c) is w_a w_b w_c."""
    rows = [l.split() for l in open(os.path.join(GOLDEN, "shape_weights.txt")) if l.strip() and not l.startswith("#")]
    assert len(rows) >= 8
    n = 16
    for r in rows:
        shape, s, first = r[0], float(r[1]), int(r[2])
        want = [float(Fraction(v)) for v in r[3:]]
        m = len(want)
        p = _uniform_params(n, shape, 1.0)
        idx, w = oracle.shape_weights(np.array([[s], [s], [s]]), p)
        assert idx.shape == (1, m ** 3)
        for c in range(m):
            for b in range(m):
                for a in range(m):
                    k = a + m * (b + m * c)
                    assert idx[0, k] == (first + a) + n * ((first + b) + n * (first + c))
                    assert w[0, k] == pytest.approx(want[a] * want[b] * want[c], abs=1e-15)


@pytest.mark.parametrize("shape", ["cic", "tsc"])
def test_partition_of_unity_and_linear_reproduction(shape):
    """Sum_i W_i = 1, and a field linear in position is reproduced exactly away from the
    periodic seam: both kernels are exact for linear functions (textbook property)."""
    n = 16
    p = _uniform_params(n, shape, 1.0)
    rng = np.random.default_rng(1)
    x = rng.uniform(3.0, 12.0, (3, 2000))
    idx, w = oracle.shape_weights(x, p)
    assert np.max(np.abs(w.sum(axis=1) - 1.0)) < 1e-14
    ic = np.arange(n ** 3)
    centres = np.stack([ic % n, (ic // n) % n, ic // n ** 2]) + 0.5
    a, b = np.array([0.3, -1.1, 2.0]), np.array([[0.7, 0.1, -0.2], [0.0, 1.3, 0.4], [-0.5, 0.2, 0.9]])
    F = a[:, None] + b @ centres
    Fp = oracle.gather(F, idx, w)
    assert np.max(np.abs(Fp - (a[:, None] + b @ x))) < 1e-12


@pytest.mark.parametrize("shape", ["cic", "tsc"])
def test_gather_deposit_adjoint(shape):
    """<b, D a> = <G b, a>: the deposit is the transpose of the gather (exact identity)."""
    n = 8
    p = _uniform_params(n, shape, 1.0)
    rng = np.random.default_rng(2)
    x = rng.uniform(0.0, n, (3, 500))
    idx, w = oracle.shape_weights(x, p)
    a = rng.standard_normal((1, 500))
    b = rng.standard_normal((1, n ** 3))
    lhs = np.sum(b * oracle.deposit(idx, w, a, n ** 3))
    rhs = np.sum(oracle.gather(b, idx, w) * a)
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)


# ---------------------------------------------------------------- gyro motion (Sec. 2 closing discussion)

def _run_single(x0, u0, E, B, p, nsteps):
    xs, us = [x0], [u0]
    x, u = x0, u0
    for _ in range(nsteps):
        x, u, _, _ = oracle.step(x, u, E, B, p)
        xs.append(x)
        us.append(u)
    return np.array(xs)[:, :, 0], np.array(us)[:, :, 0]


@pytest.mark.parametrize("ratio", [1.0, 10.0, 100.0])
def test_gyration_angle_per_step(ratio):
    """In uniform B the packet momentum rotates by 2 atan(Omega_eff dt / 2) per step with
    Omega_eff = (c_tilde/c) q B/(gamma m c) (Sec. 2: the gyro-frequency is reduced by
    c_tilde/c); clockwise about B for q > 0; the parallel momentum is untouched."""
    n = 16
    E, B = _uniform_fields(n)
    c, qomc = 1000.0, 4000.0
    u0 = np.array([[3.0], [8.0], [-2.0]])
    gamma = math.sqrt(1.0 + float(np.sum(u0 ** 2)))
    p = _uniform_params(n, "cic", ratio, dt=2.0e-3 / ratio * 10.0)
    xs, us = _run_single(np.array([[8.0], [8.0], [8.0]]), u0, E, B, p, 60)
    omega_eff = (p.c_tilde / c) * qomc * 1.0 / gamma
    want = -2.0 * math.atan(0.5 * omega_eff * p.dt)
    ang = np.arctan2(us[:-1, 1] * us[1:, 2] - us[:-1, 2] * us[1:, 1], us[:-1, 1] * us[1:, 1] + us[:-1, 2] * us[1:, 2])
    assert np.max(np.abs(ang - want)) < 1e-12 * abs(want) + 1e-15
    assert np.all(us[:, 0] == u0[0, 0])


def _circle_radius(y, z):
    """Algebraic least-squares circle fit."""
    A = np.stack([2 * y, 2 * z, np.ones_like(y)], axis=1)
    sol, *_ = np.linalg.lstsq(A, y * y + z * z, rcond=None)
    a, b, k = sol
    return math.sqrt(k + a * a + b * b), np.sqrt((y - a) ** 2 + (z - b) ** 2)


def test_gyroradius_on_grid_independent_of_ctilde():
    """Positions lie on a circle of radius r_g sqrt(1 + (Omega_eff dt/2)^2) (leapfrog chord
    geometry) with r_g = c u_perp / (q B/(m c) c)... = c u_perp/(qomc B), the same for every
    c_tilde when dt scales as 1/c_tilde (Sec. 2: gyro radius on the grid independent of c_tilde)."""
    n = 16
    E, B = _uniform_fields(n)
    c, qomc = 1000.0, 4000.0
    u0 = np.array([[0.0], [10.0], [0.0]])
    gamma = math.sqrt(101.0)
    radii = []
    for ratio in (1.0, 3.0, 10.0, 100.0):
        p = _uniform_params(n, "cic", ratio, dt=0.03 / (c / ratio))
        xs, _ = _run_single(np.array([[8.0], [8.0], [8.0]]), u0, E, B, p, 400)
        R, r_each = _circle_radius(xs[:, 1], xs[:, 2])
        assert np.max(np.abs(r_each - R)) < 1e-11 * R
        a = 0.5 * (p.c_tilde / c) * qomc / gamma * p.dt
        want = c * 10.0 / qomc * math.sqrt(1.0 + a * a)
        assert R == pytest.approx(want, rel=1e-12)
        radii.append(R)
    assert max(radii) - min(radii) < 1e-12 * radii[0]


def test_momentum_magnitude_conserved_in_pure_B():
    """|u| is conserved in a pure magnetic field: B does no work (Eq. (1)); the Boris rotation
    preserves the norm."""
    w = make_workload(1, n=8, ppc=4, nsteps=200)
    p = oracle_params(w)
    E, B = oracle_fields(w)
    x, u = w.x, w.u
    n0 = np.linalg.norm(u, axis=0)
    for _ in range(200):
        x, u, _, _ = oracle.step(x, u, E, B, p)
    assert np.max(np.abs(np.linalg.norm(u, axis=0) - n0) / n0) < 1e-14


# ---------------------------------------------------------------- E x B drift (Sec. 2, E = -(u/c) x B)

def _unwrapped(xs, box):
    d = np.diff(xs, axis=0)
    d -= box * np.round(d / box)
    return xs[0] + np.concatenate([np.zeros((1, 3)), np.cumsum(d, axis=0)])


@pytest.mark.parametrize("ratio", [1.0, 10.0, 100.0])
def test_exb_drift_on_grid(ratio):
    """A packet at rest in the frame moving with the gas drifts across the grid at
    (c_tilde/c) u_gas_perp: the frozen-in E x B velocity is the gas velocity, and the RSOL
    slows every CR advection by c_tilde/c (Sec. 2, v_eff = (c_tilde/c) v)."""
    n, U, c = 8, 1.0, 1000.0
    E, B = _uniform_fields(n, B=(1.0, 0.0, 0.0), u_gas=(0.0, U, 0.0))
    beta_e = U / c
    u0 = np.array([[0.0], [beta_e / math.sqrt(1 - beta_e ** 2)], [0.0]])
    p = _uniform_params(n, "cic", ratio, dt=0.3 / (c / ratio))
    xs, _ = _run_single(np.array([[4.0], [4.0], [4.0]]), u0, E, B, p, 200)
    xu = _unwrapped(xs, np.array([n, n, n], float))
    v = (xu[-1] - xu[0]) / (200 * p.dt)
    assert v[1] == pytest.approx((p.c_tilde / c) * U, rel=1e-6)
    assert abs(v[0]) < 1e-12 and abs(v[2]) < 1e-6 * (p.c_tilde / c) * U


def test_exb_drift_of_gyrating_guiding_centre():
    """A gyrating p = 10 packet's guiding centre R = x + (c/qomc)(u - gamma u_gas/c) x B / B^2
    drifts at (c_tilde/c) u_gas_perp; the relativistic Boris scheme reaches that value at
    second order in dt (its E x B error for gyrating relativistic packets is O(dt^2))."""
    n, U, c, qomc, ratio = 16, 1.0, 1000.0, 4000.0, 10.0
    E, B = _uniform_fields(n, B=(1.0, 0.0, 0.0), u_gas=(0.0, U, 0.0))
    errs = []
    for f in (1, 2):
        u0 = np.array([[2.0], [6.0], [7.7]])
        p = _uniform_params(n, "cic", ratio, dt=0.3 / (c / ratio) / f)
        xs, us = _run_single(np.array([[8.0], [8.0], [8.0]]), u0, E, B, p, 4000 * f)
        xu = _unwrapped(xs, np.array([n, n, n], float))
        g = np.sqrt(1.0 + np.sum(us * us, axis=1))
        # u is staggered half a step behind x; average the two neighbouring half steps
        um = 0.5 * (us[:-1] + us[1:])
        gm = 0.5 * (g[:-1] + g[1:])
        w = um - gm[:, None] * np.array([0.0, U, 0.0])[None, :] / c
        R = xu[:-1] + (c / qomc) * np.cross(w, np.array([1.0, 0.0, 0.0]))
        # least-squares slope over ~75 gyro periods averages out the residual gyro wobble of R
        t = np.arange(len(R)) * p.dt
        vy = np.polyfit(t, R[:, 1], 1)[0]
        vz = np.polyfit(t, R[:, 2], 1)[0]
        want = (p.c_tilde / c) * U
        assert abs(vz) < 1e-4 * want
        errs.append(vy / want - 1.0)
    assert abs(errs[1]) < 3e-5
    assert 3.0 < errs[0] / errs[1] < 6.0, errs


# ---------------------------------------------------------------- integrator vs continuous equations

def _analytic_field(x, c):
    """Three transverse modes along x (period 64) on B0 = x-hat; u_gas = -dB, E = -(u/c) x B."""
    ks = 2 * np.pi * np.array([1, 2, 3]) / 64.0
    amp = np.array([0.2, 0.1, 0.05])
    ph = np.array([0.3, 1.7, 4.0])
    psi = np.array([0.5, 2.0, 3.1])
    dB = np.zeros(3)
    for k, a, f, s in zip(ks, amp, ph, psi):
        prof = a * math.cos(k * x[0] + f)
        dB[1] += math.cos(s) * prof
        dB[2] += math.sin(s) * prof
    Bv = np.array([1.0, 0.0, 0.0]) + dB
    E = oracle.electric_field((-dB)[:, None], Bv[:, None], c)[:, 0]
    return E, Bv


def _convergence_ratios(pusher):
    """Position errors at T against the DOP853 solution for 200, 400, 800 steps."""
    c, qomc, ratio = 1000.0, 4000.0, 10.0
    ct = c / ratio

    def rhs(t, y):
        x, u = y[:3], y[3:]
        g = math.sqrt(1.0 + u @ u)
        E, Bv = _analytic_field(x, c)
        return np.concatenate([ct * u / g, (ct / c) * qomc * (E + np.cross(u / g, Bv))])

    x0 = np.array([10.0, 3.0, 2.0])
    u0 = np.array([5.0, 7.0, -4.0])
    T = 0.3
    ref = solve_ivp(rhs, (0.0, T), np.concatenate([x0, u0]), method="DOP853", rtol=1e-13, atol=1e-12)
    xT = ref.y[:3, -1]
    errs = []
    p = oracle.Params(64, 64, 64, 1.0, "cic", c, ct, qomc, 0.0, 1.0)
    for nsteps in (200, 400, 800):
        dt = T / nsteps
        p.dt = dt
        back = solve_ivp(rhs, (0.0, -0.5 * dt), np.concatenate([x0, u0]), method="DOP853", rtol=1e-13, atol=1e-12)
        x = x0[:, None].copy()
        u = back.y[3:, -1][:, None].copy()
        h = 0.5 * (ct / c) * qomc * dt
        for _ in range(nsteps):
            E, Bv = _analytic_field(x[:, 0], c)
            u = oracle.pic.kick(u, E[:, None], Bv[:, None], h, h, pusher)
            x = oracle.drift(x, u, p)
        d = x[:, 0] - xT
        d -= 64.0 * np.round(d / 64.0)
        errs.append(np.linalg.norm(d))
    return errs[0] / errs[1], errs[1] / errs[2], errs


@pytest.mark.parametrize("pusher", ["boris", "vay", "hc"])
def test_second_order_convergence_to_continuous_rsol_equations(pusher):
    """Kick + drift converge at second order to the continuous packet equations of Sec. 2:
    dx/dt = c_tilde u/gamma and d(u)/dt = (c_tilde/c)(q/(m c))[E + beta x B] (Eq. (11)),
    solved independently by scipy's DOP853 at tight tolerance; for the Boris, Vay and
    Higuera-Cary momentum updates alike."""
    r1, r2, errs = _convergence_ratios(pusher)
    assert 3.7 < r1 < 4.3 and 3.7 < r2 < 4.3, errs


# ---------------------------------------------------------------- c_tilde scaling laws (Secs. 2, 3)

def _run_ratio(ratio, nsteps=30):
    w = make_workload(2, n=8, ppc=2, ratio=ratio)
    p = oracle_params(w)
    E, B = oracle_fields(w)
    r = oracle.rollout(w.x, w.u, E, B, p, nsteps)
    return w, p, r


def test_step_space_invariance_under_ctilde():
    """The RSOL is a rescaling of time only (Sec. 2 after Eq. (3); Sec. 3 closing paragraph):
    with static fields and dt ~ 1/c_tilde the per-step maps depend on c_tilde dt alone, so
    states, and the exchange times c_tilde/c, are the same for every c_tilde."""
    base = None
    for ratio in (1.0, 3.0, 10.0, 30.0, 100.0):
        w, p, r = _run_ratio(ratio)
        got = (r["x"], r["u"], r["dM"] * (p.c_tilde / p.c), r["dE"] * (p.c_tilde / p.c), p.c_tilde * p.dt)
        if base is None:
            base = got
            continue
        assert np.max(np.abs(got[0] - base[0])) < 1e-11
        assert np.max(np.abs(got[1] - base[1]) / np.linalg.norm(base[1], axis=0)) < 1e-12
        assert np.max(np.abs(got[2] - base[2])) < 1e-10 * np.max(np.abs(base[2]))
        assert got[4] == pytest.approx(base[4], rel=1e-14)


def test_exchange_pinned_by_action_reaction_and_rate_invariance():
    """(a) At c_tilde = c the gas receives exactly minus the CR momentum change (textbook
    action-reaction, Sec. 2 before Eq. (12)); (b) the exchange RATE dM/dt is independent of
    c_tilde (Sec. 2: the force on the gas is the c_tilde = c one; Sec. 5, point (4)).
    Together these fix the c/c_tilde factor of Eq. (12)."""
    rates = []
    for ratio in (1.0, 10.0, 100.0):
        w = make_workload(2, n=8, ppc=2, ratio=ratio)
        p = oracle_params(w)
        E, B = oracle_fields(w)
        x1, u1, dM, dE = oracle.step(w.x, w.u, E, B, p)
        if ratio == 1.0:
            gas = dM.sum(axis=1) * p.volume
            cr = p.mass * p.c * (u1 - w.u).sum(axis=1)
            scale = p.mass * p.c * np.abs(u1 - w.u).sum()
            assert np.max(np.abs(gas + cr)) < 1e-13 * scale
        rates.append(dM / p.dt)
    for r in rates[1:]:
        assert np.max(np.abs(r - rates[0])) < 1e-10 * np.max(np.abs(rates[0]))


def test_conserved_momentum_and_energy_with_rsol():
    """rho u + (c/c_tilde) P is conserved by the exchange (Sec. 2 closing discussion), and
    likewise the energy with the packet energy M c^2 gamma (Eq. (9))."""
    w = make_workload(2, n=8, ppc=4, ratio=30.0)
    p = oracle_params(w)
    E, B = oracle_fields(w)
    x1, u1, dM, dE = oracle.step(w.x, w.u, E, B, p)
    k = p.c / p.c_tilde
    dP = p.mass * p.c * (u1 - w.u)
    g0 = np.sqrt(1 + np.sum(w.u ** 2, axis=0))
    g1 = np.sqrt(1 + np.sum(u1 ** 2, axis=0))
    dEn = p.mass * p.c ** 2 * (g1 - g0)
    # rounding bounds: the test differences the states itself, so each packet term carries
    # an error of a few ulps of M c |u| (momentum) or M c^2 gamma (energy)
    for comp in range(3):
        res = math.fsum(dM[comp] * p.volume) + k * math.fsum(dP[comp])
        assert abs(res) <= 40 * 2 ** -53 * k * p.mass * p.c * (np.abs(w.u[comp]).sum() + np.abs(u1[comp]).sum())
    res = math.fsum(dE * p.volume) + k * math.fsum(dEn)
    assert abs(res) <= 40 * 2 ** -53 * k * p.mass * p.c ** 2 * (g0.sum() + g1.sum())


# ---------------------------------------------------------------- timestep (Sec. 4)

def test_courant_dt_scaling_and_guarantees():
    """Every CR timestep limit rescales by c/c_tilde (Secs. 2 and 4): dt(c_tilde) c_tilde is
    constant; with that dt no packet moves more than C cells per step and no momentum
    rotates by more than 2 atan(C/2) per step."""
    prods = []
    for ratio in (1.0, 10.0, 30.0):
        w = make_workload(2, n=8, ppc=4, ratio=ratio)
        p = oracle_params(w)
        prods.append(p.dt * p.c_tilde)
        E, B = oracle_fields(w)
        x1, u1, _, _ = oracle.step(w.x, w.u, E, B, p)
        d = np.abs(x1 - w.x)
        d = np.minimum(d, 8.0 - d)
        assert np.max(d) <= w.courant * w.dx * (1 + 1e-12)
    assert max(prods) == pytest.approx(min(prods), rel=1e-14)
    w = make_workload(1, n=8, ppc=4)
    p = oracle_params(w)
    E, B = oracle_fields(w)
    _, u1, _, _ = oracle.step(w.x, w.u, E, B, p)
    cosang = np.sum(u1[1:] * w.u[1:], axis=0) / (np.linalg.norm(u1[1:], axis=0) * np.linalg.norm(w.u[1:], axis=0))
    assert np.max(np.arccos(np.clip(cosang, -1, 1))) <= 2 * math.atan(w.courant / 2) + 1e-9


def _rotation_angles(u0, u1):
    """Signed rotation angle of each packet's momentum about +x between two states
    (in uniform B along x the parallel component is untouched)."""
    return np.arctan2(u0[1] * u1[2] - u0[2] * u1[1], u0[1] * u1[1] + u0[2] * u1[2])


def _courant_pin_errors(ratio=10.0, qomc=4000.0):
    """Relative errors of the timestep rule against what each of its limits guarantees
    exactly when it binds (Sec. 4: dt < C / Omega_eff and dt < C dx / |v_eff|, with
    Omega_eff = (c_tilde/c) q|B|/(gamma m c) from the closing discussion of Sec. 2 and
    v_eff = c_tilde beta).  The measurements use the oracle's kick and drift, whose
    rotation angle and drift speed are pinned separately above.

    gyro: gyro-limited packets (|u| = 1 and 1.5) in a non-uniform |B| along x.  The
      packet with the smallest gamma sits at the centre of the cell with the largest |B|
      (CIC then reads that node alone), so it must rotate by exactly 2 atan(C/2) per
      step, the largest rotation of all packets.
    cell: cell-limited packets (|u| = 10 and one with |u| = 20) in uniform B: the
      fastest packet must move exactly C dx in the step.
    sign: a negative charge gives the same dt and the opposite rotation."""
    n, c, courant = 8, 1000.0, 0.3
    nc = n ** 3
    rng = np.random.default_rng(17)
    out = {}
    # gyro limit with non-uniform |B| and several gammas
    Bx = rng.uniform(0.5, 1.5, nc)
    hot = int(np.argmax(Bx))
    B = np.zeros((3, nc))
    B[0] = Bx
    E = np.zeros((3, nc))
    cells = rng.choice(nc, 40, replace=False)
    cells[0] = hot
    ix, iy, iz = cells % n, (cells // n) % n, cells // (n * n)
    x0 = np.stack([ix, iy, iz]).astype(float) + 0.5
    mag = np.where(np.arange(40) < 20, 1.0, 1.5)
    mag[0] = 1.0
    phi = rng.uniform(0, 2 * np.pi, 40)
    u0 = np.stack([np.zeros(40), mag * np.cos(phi), mag * np.sin(phi)])
    dt = oracle.courant_dt(u0, B, c, c / ratio, qomc, 1.0, courant)
    p = oracle.Params(n, n, n, 1.0, "cic", c, c / ratio, qomc, dt, 1.0)
    _, u1, _, _ = oracle.step(x0, u0, E, B, p)
    ang = _rotation_angles(u0, u1)
    want = 2.0 * math.atan(courant / 2.0)
    out["gyro"] = abs(float(np.max(np.abs(ang))) - want) / want
    out["gyro_hot"] = abs(abs(float(ang[0])) - want) / want
    out["sign_dt"] = ang[0]
    # cell limit: uniform B, |u| = 10 packets and one at |u| = 20
    Eu, Bu = _uniform_fields(n)
    m = 64
    x0 = rng.uniform(0, n, (3, m))
    d = rng.standard_normal((3, m))
    d /= np.linalg.norm(d, axis=0)
    u0 = 10.0 * d
    u0[:, 0] *= 2.0
    dt = oracle.courant_dt(u0, Bu, c, c / ratio, qomc, 1.0, courant)
    p = oracle.Params(n, n, n, 1.0, "cic", c, c / ratio, qomc, dt, 1.0)
    x1, _, _, _ = oracle.step(x0, u0, Eu, Bu, p)
    from tests.helpers import periodic_distance
    moved = periodic_distance(x1, x0, (n, n, n))
    out["cell"] = abs(float(np.max(moved)) - courant) / courant
    out["cell_fastest"] = abs(float(moved[0]) - courant) / courant
    return out


@pytest.mark.parametrize("ratio", [1.0, 10.0, 100.0])
def test_courant_dt_values_when_each_limit_binds(ratio):
    """The timestep is exactly at each limit when that limit binds (Sec. 4): the packet
    with the smallest Lorentz factor at the largest |B| rotates by 2 atan(C/2) per step
    (Omega_eff dt = C), and the fastest packet of a cell-limited set moves C dx."""
    e = _courant_pin_errors(ratio)
    assert e["gyro"] < 1e-12 and e["gyro_hot"] < 1e-12
    assert e["cell"] < 1e-12 and e["cell_fastest"] < 1e-12


def test_courant_dt_of_a_negative_charge():
    """A negative charge rotates the other way at the same gyro frequency: the same dt and
    a rotation of -2 atan(C/2) where a positive charge turns by +2 atan(C/2)."""
    pos, neg = _courant_pin_errors(10.0, 4000.0), _courant_pin_errors(10.0, -4000.0)
    assert neg["gyro"] < 1e-12 and neg["cell"] < 1e-12
    assert pos["sign_dt"] == pytest.approx(-neg["sign_dt"], rel=1e-14)
    u = np.array([[0.0, 1.0], [1.0, 0.0], [0.0, 2.0]])
    B = np.tile(np.array([[1.0], [0.0], [0.0]]), (1, 8))
    assert oracle.courant_dt(u, B, 1000.0, 100.0, -4000.0, 1.0, 0.3) == oracle.courant_dt(u, B, 1000.0, 100.0, 4000.0,
                                                                                          1.0, 0.3)


def test_planted_mistakes_fail_the_courant_pins(monkeypatch):
    """Each of these misreadings of the timestep rule fails a pin: either limit halved,
    min |B| in place of max |B|, max gamma in place of min gamma, max beta replaced by
    the mean beta."""
    pic = oracle.pic
    good = pic.courant_dt

    def variant(gyro=1.0, cell=1.0, bsel=np.max, gsel=np.min, vsel=np.max):
        def dt_rule(u, B, c, c_tilde, qomc, dx, courant, naive=False, sigma=0.0, nn=None):
            gamma = pic.lorentz_gamma(u)
            beta = np.sqrt(u[0] ** 2 + u[1] ** 2 + u[2] ** 2) / gamma
            bmag = np.sqrt(np.sum(np.asarray(B).reshape(3, -1) ** 2, axis=0))
            d_cell = cell * courant * dx / (c_tilde * vsel(beta))
            d_gyro = gyro * courant / ((c_tilde / c) * abs(qomc) * bsel(bmag) / gsel(gamma))
            return float(min(d_cell, d_gyro))
        return dt_rule

    assert max(_courant_pin_errors().values()) < 10.0  # sanity of the helper with the real rule
    for kw, key in ((dict(gyro=0.5), "gyro"), (dict(cell=0.5), "cell"), (dict(bsel=np.min), "gyro"),
                    (dict(gsel=np.max), "gyro"), (dict(vsel=np.mean), "cell")):
        with monkeypatch.context() as m:
            m.setattr(pic, "courant_dt", variant(**kw))
            m.setattr(oracle, "courant_dt", variant(**kw))
            e = _courant_pin_errors()
            assert e[key] > 1e-3, (kw, e)
    assert pic.courant_dt is good


def test_periodic_wrap_ties():
    """The periodic wrap maps every coordinate into [0, L): values already inside are
    untouched, one period is added or removed exactly where that is representable, and
    a result that rounds to L (a tiny negative coordinate) becomes 0, as does L itself."""
    L = 16.0
    tiny = 1e-300
    below = np.nextafter(L, 0.0)
    cases = [(-0.0, 0.0), (-tiny, 0.0), (0.0, 0.0), (tiny, tiny), (below, below), (L, 0.0),
             (-0.5, 15.5), (L + 0.25, 0.25), (2 * L, 0.0), (-L, 0.0), (-np.nextafter(0.0, 1.0), 0.0),
             (np.nextafter(2 * L, 0.0), np.nextafter(2 * L, 0.0) - L), (-3 * L - 2.0, L - 2.0)]
    x = np.array([a for a, _ in cases])
    got = oracle.wrap(x, L)
    want = np.array([b for _, b in cases])
    assert np.all(got >= 0.0) and np.all(got < L)
    assert np.array_equal(got, want), (got, want)
    # a drift that lands a hair below 0 leaves the packet at 0, inside the box
    p = _uniform_params(4, "cic", 1.0, dt=1.0)
    x0 = np.array([[0.0], [1.5], [2.5]])
    u = np.array([[-tiny * 1e-8], [0.0], [0.0]])
    x1 = oracle.drift(x0, u, p)
    assert x1[0, 0] == 0.0 and 0.0 <= x1[0, 0] < 4.0


def test_planted_mistake_fails_the_wrap_pin(monkeypatch):
    """Without the rule that a result equal to L becomes 0, the wrap pin fails."""
    pic = oracle.pic
    with monkeypatch.context() as m:
        def no_tie(x, length):
            y = x - length * np.floor(np.real(x) / length)
            return np.where(np.real(y) < 0, y + length, y)
        m.setattr(pic, "wrap", no_tie)
        m.setattr(oracle, "wrap", pic.wrap)
        with pytest.raises(AssertionError):
            test_periodic_wrap_ties()


# ---------------------------------------------------------------- moments (Sec. 2 packet totals)

@pytest.mark.parametrize("shape", ["cic", "tsc"])
def test_moment_totals_and_single_packet(shape):
    """Grid totals equal the packet totals N M, sum M c u, sum M c^2 gamma (partition of
    unity), and one packet at a cell centre puts (3/4)^3 (TSC) or 1 (CIC) of its mass there."""
    n = 8
    rng = np.random.default_rng(5)
    x = rng.uniform(0, n, (3, 300))
    u = rng.standard_normal((3, 300)) * 5
    p = _uniform_params(n, shape, 10.0, mass=0.37)
    rho, P, e = oracle.moments(x, u, p)
    g = np.sqrt(1 + np.sum(u * u, axis=0))
    assert rho.sum() == pytest.approx(300 * 0.37, rel=1e-13)
    assert np.allclose(P.sum(axis=1), 0.37 * 1000.0 * u.sum(axis=1), rtol=1e-12, atol=1e-9)
    assert e.sum() == pytest.approx(0.37 * 1e6 * g.sum(), rel=1e-13)
    rho1, _, _ = oracle.moments(np.array([[3.5], [4.5], [5.5]]), np.zeros((3, 1)), p)
    home = 3 + n * (4 + n * 5)
    assert rho1[home] == pytest.approx(0.37 * (0.75 ** 3 if shape == "tsc" else 1.0), rel=1e-15)


# ---------------------------------------------------------------- coupled gas (Eq. (12) closed)

_GYR = dict(n=4, c=1000.0, c_tilde=100.0, qomc=4000.0, mass=0.14, rho=2.0, T=0.01, dt0=5e-5)


def _coupled_lattice_run(dt):
    """One packet per cell on the cell centres, all with u0 = (0, 1, 0) across B = x_hat, and
    a gas of density rho carrying minus (c/c_tilde) times the CR momentum, so the total
    momentum V rho u + (c/c_tilde) P is zero.  Returns u_y + i u_z of every packet after
    T/dt coupled steps, the gas state and the Params."""
    g = _GYR
    n, nc = g["n"], g["n"] ** 3
    p = oracle.Params(n, n, n, 1.0, "cic", g["c"], g["c_tilde"], g["qomc"], dt, g["mass"])
    i = np.arange(nc)
    x = np.stack([i % n, i // n % n, i // (n * n)]).astype(float) + 0.5
    u0 = np.array([0.0, 1.0, 0.0])
    u = np.tile(u0[:, None], (1, nc))
    B = np.tile(np.array([1.0, 0.0, 0.0])[:, None], (1, nc))
    rho = np.full(nc, g["rho"])
    mom = np.tile((-(p.c / p.c_tilde) * p.mass * p.c * u0 / p.volume)[:, None], (1, nc))
    r = oracle.coupled_rollout(x, u, mom, np.zeros(nc), rho, B, p, int(round(g["T"] / dt)))
    return r["u"][1] + 1j * r["u"][2], r, p


def _coupled_gyration_errors():
    """|z - z_exact| at dt0, dt0/2, dt0/4 and of the two Richardson extrapolants 2 z(dt/2) - z(dt).

    Closed form: with the gas momentum equal to -(c/c_tilde) M c u / V in every cell,
    u_gas = mom/rho and E = -(u_gas/c) x B = (c/c_tilde)(M/(rho V)) u x B (Sec. 2, after
    Eq. (5)), so Eq. (11) becomes du/dt = qomc [M/(rho V) + (c_tilde/c)/gamma] u x B: |u| and
    gamma stay fixed and u turns about B at that rate.  For B = x_hat, u_y + i u_z advances
    by exp(-i omega t).  The scheme is first order in dt (the gas field of a step comes from
    the momentum before the kick), so the extrapolants converge at second order."""
    g = _GYR
    omega = g["qomc"] * (g["mass"] / g["rho"] + (g["c_tilde"] / g["c"]) / math.sqrt(2.0))
    exact = np.exp(-1j * omega * g["T"])
    zs = [_coupled_lattice_run(g["dt0"] / 2 ** k)[0] for k in range(3)]
    errs = [float(np.max(np.abs(z - exact))) for z in zs]
    rich = [float(np.max(np.abs(2 * zs[k + 1] - zs[k] - exact))) for k in range(2)]
    return errs, rich


def _assert_gyration_pin(errs, rich):
    assert errs[2] < 0.02
    assert 1.8 < errs[1] / errs[2] < 2.2 and 1.8 < errs[0] / errs[1] < 2.2
    assert rich[1] < 1e-3 and rich[0] / rich[1] > 3.0


def test_coupled_gyration_closed_form():
    """The coupled packet-gas system turns at qomc |B| (M/(rho V) + (c_tilde/c)/gamma): the gas
    term carries the sign and the 1/c of E = -(u/c) x B, the division by rho, and the c/c_tilde
    of Eq. (12); the packet term the c_tilde/c of Eq. (11)."""
    errs, rich = _coupled_gyration_errors()
    _assert_gyration_pin(errs, rich)
    z, r, p = _coupled_lattice_run(_GYR["dt0"] / 4)
    # the gas follows the packets exactly: every cell keeps zero total momentum
    k = p.c / p.c_tilde
    res = p.volume * r["mom"] + k * p.mass * p.c * r["u"]
    assert np.max(np.abs(res)) < 1e-12 * k * p.mass * p.c
    assert np.max(np.abs(z - z[0])) < 1e-12


def _coupled_conservation_residual():
    """Largest change of the conserved totals over 8 coupled steps of a small Alfven-wave
    workload with a non-uniform density, in units of the rounding bound of the sums."""
    w = make_workload(2, n=8, ppc=4, ratio=30.0)
    p = oracle_params(w)
    rng = np.random.default_rng(7)
    nc = w.n_cells
    rho = rng.uniform(0.5, 1.5, nc)
    B = w.B.reshape(3, -1)
    mom = rho * w.u_gas.reshape(3, -1)
    egas = rng.uniform(1.0, 2.0, nc)
    P0, E0 = oracle.conserved_totals(w.u, mom, egas, p)
    nsteps = 8
    r = oracle.coupled_rollout(w.x, w.u, mom, egas, rho, B, p, nsteps)
    P1, E1 = oracle.conserved_totals(r["u"], r["mom"], r["egas"], p)
    k = p.c / p.c_tilde
    eps = 2.0 ** -53
    # each step's deposit and the running sums round at a few ulps of the largest terms
    scale_p = k * p.mass * p.c * np.abs(w.u).sum() + p.volume * np.abs(mom).sum()
    scale_e = k * p.mass * p.c ** 2 * oracle.lorentz_gamma(w.u).sum() + p.volume * egas.sum()
    bound_p = 40 * nsteps * eps * scale_p
    bound_e = 40 * nsteps * eps * scale_e
    return max(float(np.max(np.abs(P1 - P0))) / bound_p, abs(E1 - E0) / bound_e)


def test_coupled_rollout_conserves_momentum_and_energy():
    """V sum rho u + (c/c_tilde) sum P and V sum e + (c/c_tilde) sum M c^2 gamma stay fixed to
    rounding while the gas field evolves (Sec. 2, discussion after Eq. (12))."""
    assert _coupled_conservation_residual() < 1.0


def test_planted_mistakes_fail_the_coupled_pins(monkeypatch):
    """Plausible mistakes in the coupled step each fail one of the pins above."""
    pic = oracle.pic
    good_field, good_exchange = pic.electric_field, pic.exchange

    # E with the wrong sign, and E without the division by rho
    with monkeypatch.context() as m:
        m.setattr(pic, "electric_field", lambda u, B, c: -good_field(u, B, c))
        errs, _ = _coupled_gyration_errors()
        assert errs[2] > 0.1
    with monkeypatch.context() as m:
        def no_rho(x, u, mom, egas, rho, B, p):
            E = good_field(mom, B, p.c)
            x1, u1, dM, dE = pic.step(x, u, E, B, p)
            return x1, u1, mom + dM, egas + dE
        m.setattr(pic, "coupled_step", no_rho)
        errs, _ = _coupled_gyration_errors()
        assert errs[2] > 0.1
    # exchange missing its c/c_tilde: gyration and conservation both fail
    with monkeypatch.context() as m:
        m.setattr(pic, "exchange", lambda u0, u1, p: tuple(v * (p.c_tilde / p.c) for v in good_exchange(u0, u1, p)))
        errs, _ = _coupled_gyration_errors()
        assert errs[2] > 0.1
        assert _coupled_conservation_residual() > 100.0


# ---------------------------------------------------------------- naive substitution (contrast, Secs. 1 and 5)

def _naive(p):
    return oracle.Params(p.nx, p.ny, p.nz, p.dx, p.shape, p.c, p.c_tilde, p.qomc, p.dt, p.mass, naive=True)


def _naive_force_errors(ratio=10.0):
    """Relative errors against the ratios the paper states for the naive momentum equation
    (Sec. 5, item (3)): (a) from rest in a pure E field the naive kick is (c/c_tilde)^2 times
    the RSOL one; (b) in pure B the naive rotation per step is 2 atan(Omega dt/2) with the
    unreduced Omega = q B/(gamma m c), c/c_tilde times the RSOL Omega_eff."""
    n, c, qomc = 8, 1000.0, 4000.0
    nc = n ** 3
    p = _uniform_params(n, "cic", ratio, dt=1e-5)
    x0 = np.array([[4.2], [4.7], [3.1]])
    E = np.tile(np.array([[0.3], [-0.2], [0.5]]), (1, nc))
    Z = np.zeros((3, nc))
    _, u_r, _, _ = oracle.step(x0, np.zeros((3, 1)), E, Z, p)
    _, u_n, _, _ = oracle.step(x0, np.zeros((3, 1)), E, Z, _naive(p))
    err_e = float(np.max(np.abs(u_n - (c / p.c_tilde) ** 2 * u_r)) / np.max(np.abs(u_n)))
    Ez, B = _uniform_fields(n)
    u0 = np.array([[3.0], [8.0], [-2.0]])
    gamma = math.sqrt(1.0 + float(np.sum(u0 ** 2)))
    _, us = _run_single(np.array([[4.0], [4.0], [4.0]]), u0, Ez, B, _naive(p), 20)
    want = -2.0 * math.atan(0.5 * qomc * 1.0 / gamma * p.dt)
    ang = np.arctan2(us[:-1, 1] * us[1:, 2] - us[:-1, 2] * us[1:, 1], us[:-1, 1] * us[1:, 1] + us[:-1, 2] * us[1:, 2])
    err_b = float(np.max(np.abs(ang - want)) / abs(want))
    return err_e, err_b


def test_naive_force_ratios_match_the_paper():
    err_e, err_b = _naive_force_errors()
    assert err_e < 1e-13 and err_b < 1e-12


def test_naive_equals_rsol_at_c_tilde_equal_c():
    """With c_tilde = c the naive substitution changes nothing (Sec. 1): bitwise equal."""
    w = make_workload(2, n=8, ppc=2, ratio=1.0)
    p = oracle_params(w)
    E, B = oracle_fields(w)
    a = oracle.rollout(w.x, w.u, E, B, p, 10)
    b = oracle.rollout(w.x, w.u, E, B, _naive(p), 10)
    for k in ("x", "u", "dM", "dE"):
        assert np.array_equal(a[k], b[k]), k
    for ma, mb in zip(oracle.moments(a["x"], a["u"], p), oracle.moments(b["x"], b["u"], _naive(p))):
        assert np.array_equal(ma, mb)


def _naive_gyroradius_errors():
    """Naive gyro radius on the grid: positions on a circle of radius
    (c_tilde u_perp/(qomc B)) sqrt(1 + (Omega dt/2)^2), Omega = qomc B/gamma, so it shrinks
    with c_tilde (Sec. 1: the gyro radius varies with c_tilde; Sec. 5, item (4))."""
    n = 16
    E, B = _uniform_fields(n)
    c, qomc = 1000.0, 4000.0
    u0 = np.array([[0.0], [10.0], [0.0]])
    gamma = math.sqrt(101.0)
    errs = []
    for ratio in (1.0, 10.0, 100.0):
        p = _naive(_uniform_params(n, "cic", ratio, dt=0.03 / (c / ratio)))
        xs, _ = _run_single(np.array([[8.0], [8.0], [8.0]]), u0, E, B, p, 400)
        # centred before the fit: radii down to 0.025 cells sit on coordinates near 8
        R, r_each = _circle_radius(xs[:, 1] - 8.0, xs[:, 2] - 8.0)
        a = 0.5 * qomc / gamma * p.dt
        want = p.c_tilde * 10.0 / qomc * math.sqrt(1.0 + a * a)
        errs.append(max(abs(R / want - 1.0), float(np.max(np.abs(r_each - R)) / R)))
    return max(errs)


def test_naive_gyroradius_scales_with_c_tilde():
    assert _naive_gyroradius_errors() < 1e-11


def _naive_exb_error(ratio):
    """Naive E x B drift: the force-free state (c/c_tilde) E + beta x B = 0 has
    v_eff = c_tilde beta = u_gas_perp for every c_tilde, where the RSOL drift is
    (c_tilde/c) u_gas_perp (contrast with the RSOL drift pin).  The relativistic Boris
    step keeps that state up to the change of gamma over the half kick a = h_E |E|, a
    relative error of about a^2 / 2.  Returns (relative drift error, a^2)."""
    n, U, c, qomc = 8, 1.0, 1000.0, 4000.0
    E, B = _uniform_fields(n, B=(1.0, 0.0, 0.0), u_gas=(0.0, U, 0.0))
    ct = c / ratio
    # the naive gyro frequency is not reduced: dt within both Courant limits
    p = _naive(_uniform_params(n, "cic", ratio, dt=min(0.3 / ct, 0.3 / qomc)))
    beta = U / p.c_tilde
    u0 = np.array([[0.0], [beta / math.sqrt(1 - beta ** 2)], [0.0]])
    xs, _ = _run_single(np.array([[4.0], [4.0], [4.0]]), u0, E, B, p, 200)
    xu = _unwrapped(xs, np.array([n, n, n], float))
    v = (xu[-1] - xu[0]) / (200 * p.dt)
    a = 0.5 * (c / ct) * qomc * p.dt * (U / c)
    return max(abs(v[1] / U - 1.0), abs(v[0]) / U, abs(v[2]) / U), a * a


@pytest.mark.parametrize("ratio", [1.0, 10.0, 100.0])
def test_naive_exb_drift_is_the_gas_velocity(ratio):
    err, a2 = _naive_exb_error(ratio)
    assert err < a2 + 1e-12


def _naive_moment_errors(ratio=30.0):
    """Naive CR densities for the same packets: energy, momentum and number density scale
    by (c_tilde/c)^2, (c_tilde/c)^1 and (c_tilde/c)^0 against the RSOL (true) values (Sec. 1)."""
    w = make_workload(2, n=8, ppc=2, ratio=ratio)
    p = oracle_params(w)
    r = oracle.moments(w.x, w.u, p)
    q = oracle.moments(w.x, w.u, _naive(p))
    s = p.c_tilde / p.c
    return (float(np.max(np.abs(q[0] - r[0])) / np.max(r[0])),
            float(np.max(np.abs(q[1] - s * r[1])) / np.max(np.abs(s * r[1]))),
            float(np.max(np.abs(q[2] - s * s * r[2])) / np.max(s * s * r[2])))


def test_naive_moment_scalings_match_the_paper():
    assert max(_naive_moment_errors()) < 1e-14


def _naive_exchange_residuals(ratio=30.0):
    """Naive back-reaction: the gas takes minus the change of the naive CR momentum and
    energy, so V sum dM equals minus the change of V sum of the naive moment P (and the
    same for energy), while the RSOL conserved total (with c/c_tilde and the true c) is
    not kept unless c_tilde = c.  Returns (naive momentum, naive energy, RSOL momentum)
    residuals relative to the momentum exchanged."""
    w = make_workload(2, n=8, ppc=2, ratio=ratio)
    p = _naive(oracle_params(w))
    E, B = oracle_fields(w)
    x1, u1, dM, dE = oracle.step(w.x, w.u, E, B, p)
    _, P0, e0 = oracle.moments(w.x, w.u, p)
    _, P1, e1 = oracle.moments(x1, u1, p)
    V = p.volume
    scale_p = np.abs(dM).sum() * V
    scale_e = np.abs(e1).sum() * V
    res_p = float(np.max(np.abs(V * dM.sum(axis=1) + V * (P1.sum(axis=1) - P0.sum(axis=1))))) / scale_p
    res_e = abs(V * dE.sum() + V * (e1.sum() - e0.sum())) / scale_e
    k = p.c / p.c_tilde
    rsol_total = V * dM.sum(axis=1) + k * p.mass * p.c * (u1 - w.u).sum(axis=1)
    res_r = float(np.max(np.abs(rsol_total))) / scale_p
    return res_p, res_e, res_r


def test_naive_exchange_conserves_its_own_totals_only():
    res_p, res_e, res_r = _naive_exchange_residuals()
    assert res_p < 1e-12 and res_e < 1e-13
    assert res_r > 0.1


def test_naive_breaks_step_space_invariance_and_the_timestep_gain():
    """Contrast with the RSOL invariance pin: naive rollouts at c/c_tilde = 1 and 10 with
    dt ~ 1/c_tilde differ at O(1); and where the gyro limit binds, the naive timestep at
    c_tilde < c is the c_tilde = c one (Sec. 5, item (4): no timestep gain from gyro orbits)."""
    runs = []
    for ratio in (1.0, 10.0):
        w = make_workload(2, n=8, ppc=2, ratio=ratio)
        p = _naive(oracle_params(w))
        E, B = oracle_fields(w)
        runs.append(oracle.rollout(w.x, w.u, E, B, p, 30))
    du = np.linalg.norm(runs[0]["u"] - runs[1]["u"], axis=0) / np.linalg.norm(runs[0]["u"], axis=0)
    assert np.median(du) > 0.1
    w1 = make_workload(2, n=8, ppc=2, ratio=1.0)
    w30 = make_workload(2, n=8, ppc=2, ratio=30.0)
    dt_true = oracle.courant_dt(w1.u, w1.B, w1.c, w1.c_tilde, w1.qomc, w1.dx, w1.courant)
    dt_naive = oracle.courant_dt(w30.u, w30.B, w30.c, w30.c_tilde, w30.qomc, w30.dx, w30.courant, naive=True)
    dt_rsol = oracle.courant_dt(w30.u, w30.B, w30.c, w30.c_tilde, w30.qomc, w30.dx, w30.courant)
    assert dt_naive == pytest.approx(dt_true, rel=1e-15)
    assert dt_rsol == pytest.approx(30.0 * dt_true, rel=1e-12)


def test_planted_mistakes_fail_the_naive_pins(monkeypatch):
    """Plausible mistakes in the naive constants each fail one of the naive pins."""
    pic = oracle.pic
    good = pic.naive_constants

    def variant(i):
        def f(p):
            h_e, h_b, cp, k = good(p)
            r = p.c_tilde / p.c
            return [(h_e * r * r, h_b, cp, k),      # E kick without (c/c_tilde)^2 over RSOL
                    (h_e, h_b * r, cp, k),          # rotation reduced as in RSOL
                    (h_e, h_b, cp / r, k),          # momentum/energy with the true c
                    (h_e, h_b, cp, k / r)][i]       # c/c_tilde kept on the back-reaction
        return f

    with monkeypatch.context() as m:
        m.setattr(pic, "naive_constants", variant(0))
        assert max(_naive_force_errors()) > 1e-3 and _naive_exb_error(10.0)[0] > 1e-3
    with monkeypatch.context() as m:
        m.setattr(pic, "naive_constants", variant(1))
        assert _naive_force_errors()[1] > 1e-3 and _naive_gyroradius_errors() > 1e-3
    with monkeypatch.context() as m:
        m.setattr(pic, "naive_constants", variant(2))
        assert max(_naive_moment_errors()) > 1e-3
    with monkeypatch.context() as m:
        m.setattr(pic, "naive_constants", variant(3))
        assert max(_naive_exchange_residuals()[:2]) > 1e-3


# ---------------------------------------------------------------- catastrophic losses (Secs. 2 and 4)

def _loss_gyration_errors():
    """Weight of a gyrating packet in uniform B and uniform n_n.  B does no work, so beta is
    constant and the weight after N steps is exp(-sigma n_n L) with L = N c_tilde beta dt
    the path length on the grid (also measured from the positions).  (a) With dt ~ 1/c_tilde
    the weight is the same for every c_tilde: the loss per distance does not depend on
    c_tilde (Sec. 2, closing discussion).  (b) At a fixed dt the weight after a physical
    time T is exp(-(c_tilde/c) sigma c beta n_n T): the loss rate is slowed by c_tilde/c.
    Returns the largest relative error of the weight against these closed forms."""
    n, c, qomc, sigma, nn0 = 16, 1000.0, 4000.0, 0.05, 1.3
    E, B = _uniform_fields(n)
    nn = np.full(n ** 3, nn0)
    u0 = np.array([[3.0], [8.0], [-2.0]])
    beta = math.sqrt(float(np.sum(u0 ** 2))) / math.sqrt(1.0 + float(np.sum(u0 ** 2)))
    errs, ws = [], []
    for ratio in (1.0, 10.0, 100.0):
        p = _uniform_params(n, "cic", ratio, dt=0.3 / (c / ratio))  # 0.3 cells per step
        x, u, w = np.array([[8.0], [8.0], [8.0]]), u0, np.ones(1)
        L = 0.0
        for _ in range(60):
            x1, u, w, _, _ = oracle.step_with_losses(x, u, w, E, B, nn, sigma, p)
            d = x1 - x
            d -= n * np.round(d / n)
            L += float(np.sqrt(np.sum(d * d)))
            x = x1
        want = math.exp(-sigma * nn0 * 60 * p.c_tilde * beta * p.dt)
        errs += [abs(w[0] / want - 1.0), abs(L / (60 * p.c_tilde * beta * p.dt) - 1.0)]
        ws.append(w[0])
    errs.append(max(ws) / min(ws) - 1.0)
    for ratio in (1.0, 10.0):
        p = _uniform_params(n, "cic", ratio, dt=1e-4)
        x, u, w = np.array([[8.0], [8.0], [8.0]]), u0, np.ones(1)
        for _ in range(50):
            x, u, w, _, _ = oracle.step_with_losses(x, u, w, E, B, nn, sigma, p)
        want = math.exp(-(p.c_tilde / c) * sigma * c * beta * nn0 * 50 * p.dt)
        errs.append(abs(w[0] / want - 1.0))
    return max(errs)


def test_loss_per_distance_independent_of_c_tilde():
    assert _loss_gyration_errors() < 1e-12


def _loss_density_sample_error(shape):
    """A packet on a straight path (no fields) through a nucleon density that is linear
    along x on the cell centres, n_n = a + b x (reproduced exactly by CIC and TSC): the
    weight is exp(-sigma sum_n n_n(x^n) dl), the density taken at the start of every step,
    whose closed form is sigma [(a + b x0) N dl + b dl^2 N (N-1)/2]."""
    n, sigma, a, b = 32, 0.05, 1.0, 0.05
    p = _uniform_params(n, shape, 10.0, dt=3e-3)
    Z = np.zeros((3, n ** 3))
    i = np.arange(n ** 3)
    nn = a + b * ((i % n) + 0.5)
    uz = 0.8
    u = np.array([[uz], [0.0], [0.0]])
    beta = uz / math.sqrt(1 + uz * uz)
    x, w = np.array([[6.3], [9.5], [11.2]]), np.ones(1)
    N = 40
    for _ in range(N):
        x, u, w, _, _ = oracle.pic.step_with_losses(x, u, w, Z, Z, nn, sigma, p)
    dl = p.c_tilde * beta * p.dt
    want = math.exp(-sigma * ((a + b * 6.3) * N * dl + b * dl * dl * N * (N - 1) / 2))
    return abs(w[0] / want - 1.0)


@pytest.mark.parametrize("shape", ["cic", "tsc"])
def test_loss_takes_the_density_at_the_step_start(shape):
    assert _loss_density_sample_error(shape) < 1e-12


def _loss_conservation_residual():
    """Over 8 steps with strong losses the gas takes both the Lorentz-force exchange and
    what the losses remove: V sum dM + (c/c_tilde) sum_j w_j M c u_j and the energy total
    stay fixed to rounding (Sec. 2: conserved rho u + (c/c_tilde) P)."""
    w = make_workload(2, n=8, ppc=4, ratio=30.0)
    p = oracle_params(w)
    E, B = oracle_fields(w)
    nn, _, wt = loss_state(w)
    sigma = 2.0
    r = oracle.rollout_with_losses(w.x, w.u, wt, E, B, nn, sigma, p, 8)
    zero3, zero = np.zeros((3, w.n_cells)), np.zeros(w.n_cells)
    P0, E0 = oracle.conserved_totals(w.u, zero3, zero, p, w=wt)
    P1, E1 = oracle.conserved_totals(r["u"], r["dM_sum"], r["dE_sum"], p, w=r["w"])
    k = p.c / p.c_tilde
    eps = 2.0 ** -53
    scale_p = k * p.mass * p.c * np.abs(w.u).sum()
    scale_e = k * p.mass * p.c ** 2 * oracle.lorentz_gamma(w.u).sum()
    lost = 1.0 - float(r["w"].mean())
    return max(float(np.max(np.abs(P1 - P0))) / (40 * 8 * eps * scale_p),
               abs(E1 - E0) / (40 * 8 * eps * scale_e)), lost


def test_losses_hand_what_they_remove_to_the_gas():
    res, lost = _loss_conservation_residual()
    assert res < 1.0 and lost > 0.01


def _loss_courant_error():
    """Where the loss limit binds, one step of the Courant dt removes exactly C e-folds of
    the fastest-losing packet (Sec. 4: dt < C N_j/|dN_j/dt|), and that dt grows as c/c_tilde."""
    w = make_workload(2, n=8, ppc=2, ratio=30.0)
    nn, _, _ = loss_state(w)
    sigma = 50.0
    dts, errs = [], []
    for ratio in (1.0, 30.0):
        ct = w.c / ratio
        dt = oracle.courant_dt(w.u, w.B, w.c, ct, w.qomc, w.dx, w.courant, sigma=sigma, nn=nn)
        p = oracle.Params(w.nx, w.ny, w.nz, w.dx, w.shape, w.c, ct, w.qomc, dt, w.mass)
        g = oracle.lorentz_gamma(w.u)
        j = int(np.argmax(np.linalg.norm(w.u, axis=0) / g))
        f = oracle.pic.loss_factor(w.u[:, j:j + 1], np.array([nn.max()]), sigma, p)
        dts.append(dt)
        errs.append(abs(-math.log(float(f[0])) / w.courant - 1.0))
    return max(errs + [abs(dts[1] / dts[0] / 30.0 - 1.0)])


def test_loss_timestep_limit():
    assert _loss_courant_error() < 1e-12


def test_zero_cross_section_is_the_loss_free_step():
    w = make_workload(2, n=8, ppc=2)
    p = oracle_params(w)
    E, B = oracle_fields(w)
    nn, _, wt = loss_state(w)
    a = oracle.step(w.x, w.u, E, B, p)
    b = oracle.step_with_losses(w.x, w.u, wt, E, B, nn, 0.0, p)
    assert np.array_equal(b[2], wt)
    for ka, kb in ((0, 0), (1, 1), (2, 3), (3, 4)):
        assert np.allclose(a[ka], b[kb], rtol=1e-15, atol=0), ka


def test_planted_mistakes_fail_the_loss_pins(monkeypatch):
    """Plausible mistakes in the loss stage each fail one of the loss pins."""
    pic = oracle.pic
    good_factor, good_step = pic.loss_factor, pic.step_with_losses
    with monkeypatch.context() as m:
        # rate without the c_tilde/c reduction
        m.setattr(pic, "loss_factor", lambda u, nn, s, p: good_factor(u, nn, s * p.c / p.c_tilde, p))
        assert _loss_gyration_errors() > 1e-3 and _loss_courant_error() > 1e-3
    with monkeypatch.context() as m:
        # density taken after the drift
        def late(x, u, w, E, B, nn, sigma, p):
            x1, u1, _, dM, dE = good_step(x, u, w, E, B, nn, 0.0, p)
            idx, wts = pic.shape_weights(x1, p)
            return x1, u1, w * good_factor(u1, pic.gather(nn[None], idx, wts)[0], sigma, p), dM, dE
        m.setattr(pic, "step_with_losses", late)
        assert _loss_density_sample_error("cic") > 1e-4
    with monkeypatch.context() as m:
        # the removed packet totals not handed to the gas
        m.setattr(pic, "exchange_weighted", lambda u0, w0, u1, w1, p: tuple(w1 * v for v in pic.exchange(u0, u1, p)))
        assert _loss_conservation_residual()[0] > 100.0


# ---------------------------------------------------------------- alternative pushers (Vay, Higuera-Cary)

def _with_pusher(p, pusher):
    return oracle.Params(p.nx, p.ny, p.nz, p.dx, p.shape, p.c, p.c_tilde, p.qomc, p.dt, p.mass, pusher=pusher)


def _force_free_drift(pusher, ratio=10.0):
    """Largest momentum change over 200 steps of a packet in the force-free E x B state
    E + beta x B = 0 (beta = u_gas/c for E = -(u_gas/c) x B): the Vay and Higuera-Cary
    schemes keep it exactly by construction, Boris only up to the gamma change over its
    half kick.  Returned relative to |u|."""
    n, U, c = 8, 1.0, 1000.0
    E, B = _uniform_fields(n, B=(1.0, 0.0, 0.0), u_gas=(0.0, U, 0.0))
    beta = U / c
    u0 = np.array([[0.0], [beta / math.sqrt(1 - beta ** 2)], [0.0]])
    p = _with_pusher(_uniform_params(n, "cic", ratio, dt=0.3 / (c / ratio)), pusher)
    _, us = _run_single(np.array([[4.0], [4.0], [4.0]]), u0, E, B, p, 200)
    return float(np.max(np.abs(us - us[0]))) / float(u0[1, 0])


def test_vay_and_higuera_cary_keep_the_exb_drift_exactly():
    for pusher in ("vay", "hc"):
        assert _force_free_drift(pusher) < 1e-13, pusher
    assert _force_free_drift("boris") > 1e-8


def _pure_b_rotation_errors(pusher):
    """In uniform B: |u| is kept (B does no work).  Vay rotates by Boris' angle
    2 atan(h_b B/gamma).  Higuera-Cary rotates by 2 atan(h_b B/gamma_a), where gamma_a is the
    Lorentz factor of the average of the momenta before and after the step (its implicit
    velocity average), checked from the states themselves."""
    n = 16
    E, B = _uniform_fields(n)
    u0 = np.array([[3.0], [8.0], [-2.0]])
    p = _with_pusher(_uniform_params(n, "cic", 10.0, dt=2e-3), pusher)
    _, us = _run_single(np.array([[8.0], [8.0], [8.0]]), u0, E, B, p, 40)
    nrm = np.linalg.norm(us, axis=1)
    hb = 0.5 * (p.c_tilde / p.c) * p.qomc * p.dt
    ang = np.arctan2(us[:-1, 1] * us[1:, 2] - us[:-1, 2] * us[1:, 1], us[:-1, 1] * us[1:, 1] + us[:-1, 2] * us[1:, 2])
    if pusher == "hc":
        avg = 0.5 * (us[:-1] + us[1:])
        ga = np.sqrt(1.0 + np.sum(avg * avg, axis=1))
        want = -2.0 * np.arctan(hb * 1.0 / ga)
    else:
        want = -2.0 * np.arctan(hb * 1.0 / np.sqrt(1.0 + nrm[:-1] ** 2))
    return max(float(np.max(np.abs(nrm - nrm[0]))) / nrm[0], float(np.max(np.abs(ang - want) / np.abs(want))))


@pytest.mark.parametrize("pusher", ["vay", "hc"])
def test_pusher_rotation_in_pure_b(pusher):
    assert _pure_b_rotation_errors(pusher) < 1e-12


@pytest.mark.parametrize("pusher", ["vay", "hc"])
def test_pusher_step_space_invariance(pusher):
    """The RSOL stays a rescaling of time with any pusher: the per-step maps depend on
    c_tilde dt alone (the c_tilde/c of Eq. (11) enters only through h = (c_tilde/c) qomc dt/2)."""
    base = None
    for ratio in (1.0, 10.0, 100.0):
        w = make_workload(2, n=8, ppc=2, ratio=ratio)
        p = _with_pusher(oracle_params(w), pusher)
        E, B = oracle_fields(w)
        r = oracle.rollout(w.x, w.u, E, B, p, 30)
        if base is None:
            base = r
            continue
        assert np.max(np.abs(r["x"] - base["x"])) < 1e-11
        assert np.max(np.abs(r["u"] - base["u"]) / np.linalg.norm(base["u"], axis=0)) < 1e-12


def test_planted_mistakes_fail_the_pusher_pins(monkeypatch):
    """Plausible mistakes in the Vay and Higuera-Cary updates each fail a pusher pin."""
    pic = oracle.pic
    good_gamma = pic._implicit_gamma
    with monkeypatch.context() as m:
        # Vay without the magnetic half of its first stage, u' = u + 2 h E
        def vay_short(u, E, B, h, hb):
            up = u + 2.0 * h * E
            tau = hb * B
            t = tau / good_gamma(up, tau)
            sv = 1.0 / (1.0 + np.sum(t * t, axis=0))
            return sv * (up + np.sum(up * t, axis=0) * t + np.cross(up, t, axis=0))
        m.setattr(pic, "vay_kick", vay_short)
        assert _pure_b_rotation_errors("vay") > 1e-6 and _force_free_drift("vay") > 1e-8
    with monkeypatch.context() as m:
        # rotation with gamma of the rotated vector itself (the Boris choice) instead of the implicit root
        m.setattr(pic, "_implicit_gamma", lambda v, tau: np.sqrt(1.0 + v[0] ** 2 + v[1] ** 2 + v[2] ** 2))
        assert _force_free_drift("hc") > 1e-8 and _force_free_drift("vay") > 1e-8
    with monkeypatch.context() as m:
        # Higuera-Cary without the final u+ x t
        def hc_short(u, E, B, h, hb):
            um = u + h * E
            tau = hb * B
            t = tau / good_gamma(um, tau)
            sv = 1.0 / (1.0 + np.sum(t * t, axis=0))
            return sv * (um + np.sum(um * t, axis=0) * t + np.cross(um, t, axis=0)) + h * E
        m.setattr(pic, "hc_kick", hc_short)
        assert _pure_b_rotation_errors("hc") > 1e-6


# ---------------------------------------------------------------- reference gradients

def test_complex_step_gradient_matches_central_difference_and_full_rerun():
    """The structured complex-step gradient agrees with (a) an unstructured complex step of the
    whole rollout and (b) the exact-summation central difference, on a small case."""
    w = make_workload(5, n=4, ppc=2, nsteps=6)
    p = oracle_params(w)
    E, B = oracle_fields(w)
    coords = [("E", 1, 5), ("B", 2, 17), ("u", 0, 3), ("u", 2, 60), ("B", 1, 40)]
    cells = [c for k, _, c in coords if k != "u"]
    touch = adjoint.packets_touching(w.x, w.u, E, B, p, 6, cells)
    g_cs, L0 = adjoint.complex_step_grad(w.x, w.u, E, B, p, 6, w.target.reshape(3, -1), coords, touch)
    g_fd = adjoint.central_fd_grad(w.x, w.u, E, B, p, 6, w.target.reshape(3, -1), coords, touch)
    h = 1e-30
    for (kind, comp, where), gc, gf in zip(coords, g_cs, g_fd):
        Ec, Bc, uc = E.astype(complex), B.astype(complex), w.u.astype(complex)
        {"E": Ec, "B": Bc, "u": uc}[kind][comp, where] += 1j * h
        P = adjoint.final_momentum_density(w.x.astype(complex), uc, Ec, Bc, p, 6)
        full = np.imag(adjoint.momentum_loss(P, w.target.reshape(3, -1))) / h
        assert gc == pytest.approx(full, rel=1e-9, abs=1e-14 * abs(L0))
        assert gf == pytest.approx(gc, rel=1e-5, abs=1e-9 * abs(L0))
