"""Plain float64 reference of one RSOL MHD-PIC step (gather, kick, exchange
deposit, drift), the CR moments and the timestep rule.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Every array operation
here is written to accept complex128 as well as float64 so that the same code
yields complex-step derivatives; floors and the periodic wrap act on the real
part only.

Layouts: grid quantities are (C, n_cells) or (C, nz, ny, nx) with x fastest,
cell = ix + nx*(iy + ny*iz); packets are (3, Np).  Fields are cell-centred:
the node of cell i sits at (i + 1/2) dx.
"""

from __future__ import annotations

from dataclasses import dataclass

import numpy as np


@dataclass
class Params:
    """Run parameters of the packet integrator (all in the workload's code units)."""
    nx: int
    ny: int
    nz: int
    dx: float
    shape: str          # "cic" or "tsc": the spatial kernel W of the packet decomposition
    c: float            # true speed of light
    c_tilde: float      # reduced speed of light
    qomc: float         # q / (m_s c) of the CR species
    dt: float
    mass: float         # packet mass weight M_j = N_j <m_s>
    naive: bool = False  # naive substitution of c by c_tilde (contrast mode, see naive_constants)
    pusher: str = "boris"  # momentum update: "boris", "vay" or "hc" (Higuera-Cary)

    @property
    def n_cells(self):
        return self.nx * self.ny * self.nz

    @property
    def volume(self):
        return self.dx ** 3


def lorentz_gamma(u):
    """True Lorentz factor of a packet from u = gamma*beta (Sec. 2, Eqs. (7)-(8)):
    gamma = 1/sqrt(1 - beta.beta) = sqrt(1 + u.u)."""
    return np.sqrt(1.0 + u[0] * u[0] + u[1] * u[1] + u[2] * u[2])


def electric_field(u_gas, B, c):
    """Ideal-MHD electric field E = -(u/c) x B with the TRUE c (Sec. 2, the
    definition following Eq. (5))."""
    return -np.cross(u_gas, B, axis=0) / c


def courant_dt(u, B, c, c_tilde, qomc, dx, courant, naive=False, sigma=0.0, nn=None):
    """One global RSOL timestep (Sec. 4, timestep constraints; Sec. 2, closing
    discussion).  Gyro limit dt < C / Omega_eff with Omega_eff = (c_tilde/c) q|B|/(gamma m c)
    and cell-crossing limit dt < C dx / |v_eff| with v_eff = c_tilde beta.
    Both carry the factor c/c_tilde relative to c_tilde = c.  Under the naive
    substitution the gyro frequency is not reduced (Sec. 5, items (3)-(4)):
    Omega = q|B|/(gamma m c)."""
    gamma = lorentz_gamma(u)
    beta = np.sqrt(u[0] ** 2 + u[1] ** 2 + u[2] ** 2) / gamma
    bmag = np.sqrt(np.sum(np.asarray(B).reshape(3, -1) ** 2, axis=0))
    dt_cell = courant * dx / (c_tilde * np.max(beta))
    # the limit concerns the gyro frequency's magnitude, whatever the sign of the charge
    omega_max = (1.0 if naive else c_tilde / c) * abs(qomc) * np.max(bmag) / np.min(gamma)
    dt_gyro = courant / omega_max
    dt = min(dt_cell, dt_gyro)
    if sigma > 0 and nn is not None and np.max(nn) > 0 and np.max(beta) > 0:
        # catastrophic losses (Sec. 4): dt < C N_j/|dN_j/dt| with the (c_tilde/c)-reduced
        # rate (c_tilde/c) sigma c beta n_n, at the largest beta and n_n
        dt = min(dt, courant / ((c_tilde / c) * sigma * c * np.max(beta) * np.max(nn)))
    return float(dt)


def _axis_weights(s, n, shape):
    """Node indices and weights along one axis for a position s = x/dx.

    CIC: nodes i0, i0+1 with i0 = floor(s - 1/2), weights (1-f, f).
    TSC: nodes i-1, i, i+1 around the home cell i = floor(s), with
    d = s - i - 1/2, weights (1/2 (1/2-d)^2, 3/4 - d^2, 1/2 (1/2+d)^2).
    These are the standard Hockney-Eastwood assignment functions standing in
    for the paper's spatial kernel W of the packet decomposition (Sec. 2, Eq. (4)).
    """
    if shape == "cic":
        sp = s - 0.5
        i0 = np.floor(np.real(sp)).astype(np.int64)
        f = sp - i0
        nodes = [i0, i0 + 1]
        wts = [1.0 - f, f]
    elif shape == "tsc":
        i = np.floor(np.real(s)).astype(np.int64)
        d = s - i - 0.5
        nodes = [i - 1, i, i + 1]
        wts = [0.5 * (0.5 - d) ** 2, 0.75 - d * d, 0.5 * (0.5 + d) ** 2]
    else:
        raise ValueError(shape)
    return [np.mod(a, n) for a in nodes], wts


def shape_weights(x, p: Params):
    """Flat node indices (Np, K) and tensor-product weights (Np, K) of every
    packet, K = 8 (CIC) or 27 (TSC); column k = a + m*(b + m*c) for the x, y, z
    offsets a, b, c of an m-point stencil."""
    ix, wx = _axis_weights(x[0] / p.dx, p.nx, p.shape)
    iy, wy = _axis_weights(x[1] / p.dx, p.ny, p.shape)
    iz, wz = _axis_weights(x[2] / p.dx, p.nz, p.shape)
    idx, w = [], []
    for c in range(len(iz)):
        for b in range(len(iy)):
            for a in range(len(ix)):
                idx.append(ix[a] + p.nx * (iy[b] + p.ny * iz[c]))
                w.append(wx[a] * wy[b] * wz[c])
    return np.stack(idx, axis=1), np.stack(w, axis=1)


def gather(F, idx, w):
    """Field at each packet, F_p = sum_i W(x_p - x_i) F_i (the kernel-weighted
    field average that Eq. (5) evaluates at the packet, Sec. 2).
    F is (C, n_cells); returns (C, Np)."""
    return np.einsum("cnk,nk->cn", F[:, idx], w)


def deposit(idx, w, vals, n_cells):
    """Scatter sum_j W(x_j - x_i) vals_j onto the grid (the sum over packets in
    Eq. (12) and in the moments of Sec. 2).  vals is (C, Np); returns (C, n_cells)."""
    flat = idx.ravel()
    out = []
    for v in vals:
        contrib = (w * v[:, None]).ravel()
        if np.iscomplexobj(contrib):
            r = np.bincount(flat, weights=contrib.real, minlength=n_cells)
            i = np.bincount(flat, weights=contrib.imag, minlength=n_cells)
            out.append(r + 1j * i)
        else:
            out.append(np.bincount(flat, weights=contrib, minlength=n_cells))
    return np.stack(out)


def boris_kick(u, Ep, Bp, h, h_b=None):
    """Advance u = gamma*beta by one step of Eq. (11),
    d(gamma beta)/dt = (c_tilde/c) (q/(m c)) [E + beta x B],
    with the relativistic Boris scheme (half electric kick, magnetic rotation
    about B with gamma taken after the half kick, half electric kick).
    h = (c_tilde/c) (q/(m c)) dt / 2; returns u at the next half step.
    With h_b given, the electric half kick is h E and the rotation uses h_b: the
    same scheme for du/dt = (2h/dt) E + (2h_b/dt) beta x B (the naive equation)."""
    if h_b is None:
        h_b = h
    um = u + h * Ep
    gm = lorentz_gamma(um)
    t = (h_b / gm) * Bp
    tt = t[0] * t[0] + t[1] * t[1] + t[2] * t[2]
    s = 2.0 * t / (1.0 + tt)
    up = um + np.cross(um, t, axis=0)
    uplus = um + np.cross(up, s, axis=0)
    return uplus + h * Ep


def _implicit_gamma(v, tau):
    """Lorentz factor after the magnetic rotation of the Vay and Higuera-Cary schemes for
    the vector v being rotated: the positive root of
    gamma^4 - sigma gamma^2 - (tau.tau + (v.tau)^2) = 0, sigma = 1 + v.v - tau.tau."""
    tt = tau[0] * tau[0] + tau[1] * tau[1] + tau[2] * tau[2]
    vt = v[0] * tau[0] + v[1] * tau[1] + v[2] * tau[2]
    sig = 1.0 + v[0] * v[0] + v[1] * v[1] + v[2] * v[2] - tt
    return np.sqrt(0.5 * (sig + np.sqrt(sig * sig + 4.0 * (tt + vt * vt))))


def vay_kick(u, Ep, Bp, h, h_b):
    """The relativistic pusher of Vay (Phys. Plasmas 15, 056701, 2008) for
    du/dt = (2h/dt) E + (2h_b/dt) beta x B: u' = u + 2h E + h_b (u/gamma) x B; tau = h_b B;
    the new gamma solves the quartic of the implicit velocity average; t = tau/gamma,
    s = 1/(1 + t.t), u_new = s [u' + (u'.t) t + u' x t].  A particle in the force-free
    E x B drift keeps its momentum exactly."""
    g = lorentz_gamma(u)
    up = u + 2.0 * h * Ep + h_b * np.cross(u / g, Bp, axis=0)
    tau = h_b * Bp
    gn = _implicit_gamma(up, tau)
    t = tau / gn
    s = 1.0 / (1.0 + t[0] * t[0] + t[1] * t[1] + t[2] * t[2])
    upt = up[0] * t[0] + up[1] * t[1] + up[2] * t[2]
    return s * (up + upt * t + np.cross(up, t, axis=0))


def hc_kick(u, Ep, Bp, h, h_b):
    """The relativistic pusher of Higuera and Cary (Phys. Plasmas 24, 052104, 2017) for the
    same equation: half electric kick u- = u + h E; the rotation uses the Lorentz factor of
    the implicit velocity average (the quartic of the Vay scheme, applied to u-), t = tau/gamma,
    s = 1/(1 + t.t), u+ = s [u- + (u-.t) t + u- x t]; then u_new = u+ + h E + u+ x t."""
    um = u + h * Ep
    tau = h_b * Bp
    gn = _implicit_gamma(um, tau)
    t = tau / gn
    s = 1.0 / (1.0 + t[0] * t[0] + t[1] * t[1] + t[2] * t[2])
    umt = um[0] * t[0] + um[1] * t[1] + um[2] * t[2]
    uplus = s * (um + umt * t + np.cross(um, t, axis=0))
    return uplus + h * Ep + np.cross(uplus, t, axis=0)


def kick(u, Ep, Bp, h, h_b, pusher="boris"):
    """The momentum update of one step with the chosen pusher."""
    if pusher == "boris":
        return boris_kick(u, Ep, Bp, h, h_b)
    if pusher == "vay":
        return vay_kick(u, Ep, Bp, h, h_b)
    if pusher == "hc":
        return hc_kick(u, Ep, Bp, h, h_b)
    raise ValueError(f"unknown pusher {pusher}")


def naive_constants(p: Params):
    """Constants of the naive substitution of c by c_tilde (the prior approach the
    paper contrasts with, Sec. 1 and Sec. 5): the Lorentz factor is formed with
    c_tilde, gamma = c_tilde / sqrt(c_tilde^2 - v^2), so u = gamma v / c_tilde; the
    momentum equation is d_t(gamma v_eff) = (q/(m c)) (c E + v_eff x B) (Sec. 5, item
    (3)), i.e. du/dt = (q/(m c)) [(c/c_tilde) E + beta x B]; the packet momentum and
    energy are M c_tilde u and M c_tilde^2 gamma (Sec. 5, item (1); Sec. 1, the c_tilde^1
    and c_tilde^2 of the CR momentum and energy densities), and the gas takes their
    change with no c/c_tilde factor.
    Returns (electric half kick, magnetic half kick, speed in P and energy, exchange factor)."""
    h_e = 0.5 * (p.c / p.c_tilde) * p.qomc * p.dt
    h_b = 0.5 * p.qomc * p.dt
    return h_e, h_b, p.c_tilde, 1.0


def rsol_constants(p: Params):
    """The RSOL counterparts: both half kicks (c_tilde/c) (q/(m c)) dt / 2 (Eq. (11)),
    P_j = M c u and energy M c^2 gamma with the true c (Eqs. (9)-(10)), and the c/c_tilde
    of the back-reaction (Eq. (12))."""
    h = 0.5 * (p.c_tilde / p.c) * p.qomc * p.dt
    return h, h, p.c, p.c / p.c_tilde


def mode_constants(p: Params):
    return naive_constants(p) if p.naive else rsol_constants(p)


def exchange(u_old, u_new, p: Params):
    """Momentum and energy each packet hands to the gas over one step.
    Momentum: Eq. (12), d(rho u)/dt = -sum_j (1/V_j)(c/c_tilde) d_t P_j with
    P_j = M_j c u_j (Sec. 2, Eq. (10) and the packet totals).  Energy: the
    same equal-and-opposite rule applied to the packet energy M_j c^2 gamma_j
    (Eq. (9)).  Naive mode: P_j = M_j c_tilde u_j, energy M_j c_tilde^2 gamma_j and
    no c/c_tilde factor (naive_constants).
    Returns (dP (3, Np), dE (Np)) per packet, before weighting."""
    _, _, cp, k = mode_constants(p)
    f = -k * p.mass * cp
    dP = f * (u_new - u_old)
    dE = f * cp * (lorentz_gamma(u_new) - lorentz_gamma(u_old))
    return dP, dE


def loss_factor(u_new, nn_p, sigma, p: Params):
    """Fraction of a packet kept over one step under catastrophic losses (Sec. 2, the
    collisional terms): every packet total psi = (N, M, E, P) decays as
    d_t psi = -(c_tilde/c) <sigma v> n_n psi, with the reduced rate.  Here
    <sigma v> = sigma c beta for a constant cross-section sigma, beta from the step's
    momentum u^{n+1/2}, and n_n the nucleon density at the packet at x^n; the decay over
    the step is integrated exactly with that frozen rate.  The exponent is then
    sigma n_n times the step's drift length c_tilde beta dt: the loss per distance
    travelled does not depend on c_tilde (Sec. 2, closing discussion)."""
    beta = np.sqrt(u_new[0] ** 2 + u_new[1] ** 2 + u_new[2] ** 2) / lorentz_gamma(u_new)
    return np.exp(-(p.c_tilde / p.c) * sigma * p.c * beta * nn_p * p.dt)


def exchange_weighted(u_old, w_old, u_new, w_new, p: Params):
    """exchange() for packets whose weight changes over the step: the gas takes the change
    of the packet totals P_j = w_j M c u_j and w_j M c^2 gamma_j (Eq. (12) and its energy
    reading), so what the losses remove is handed to the gas as well."""
    _, _, cp, k = mode_constants(p)
    f = -k * p.mass * cp
    dP = f * (w_new * u_new - w_old * u_old)
    dE = f * cp * (w_new * lorentz_gamma(u_new) - w_old * lorentz_gamma(u_old))
    return dP, dE


def step_with_losses(x, u, w, E, B, nn, sigma, p: Params):
    """One packet step with catastrophic losses: gather E, B and the nucleon density nn
    (n_cells,) at x^n, kick, reduce the weight w (Np,) by loss_factor, deposit the change
    of the weighted packet totals at x^n, drift.
    Returns (x^{n+1}, u^{n+1/2}, w^{n+1}, dM, dE)."""
    idx, wts = shape_weights(x, p)
    Ep = gather(E, idx, wts)
    Bp = gather(B, idx, wts)
    nn_p = gather(np.asarray(nn)[None], idx, wts)[0]
    h_e, h_b, _, _ = mode_constants(p)
    u_new = kick(u, Ep, Bp, h_e, h_b, p.pusher)
    w_new = w * loss_factor(u_new, nn_p, sigma, p)
    dP, dEn = exchange_weighted(u, w, u_new, w_new, p)
    dep = deposit(idx, wts, np.concatenate([dP, dEn[None]]), p.n_cells) / p.volume
    x_new = drift(x, u_new, p)
    return x_new, u_new, w_new, dep[0:3], dep[3]


def rollout_with_losses(x, u, w, E, B, nn, sigma, p: Params, nsteps):
    """nsteps steps with losses; returns the final state and weights and the exchange
    summed over the steps."""
    dM_sum = np.zeros((3, p.n_cells))
    dE_sum = np.zeros(p.n_cells)
    for _ in range(nsteps):
        x, u, w, dM, dE = step_with_losses(x, u, w, E, B, nn, sigma, p)
        dM_sum = dM_sum + dM
        dE_sum = dE_sum + dE
    return dict(x=x, u=u, w=w, dM_sum=dM_sum, dE_sum=dE_sum)


def wrap(x, length):
    """Periodic wrap into [0, length): x - length floor(x/length); a result equal to
    length maps to 0, and so does a tiny negative x whose quotient underflows to -0
    (it would otherwise stay negative)."""
    y = x - length * np.floor(np.real(x) / length)
    y = np.where(np.real(y) < 0, y + length, y)
    return np.where(np.real(y) >= length, y - length, y)


def drift(x, u_new, p: Params):
    """Position update of Sec. 2: d<x>/dt = (c_tilde/c) <v> = c_tilde beta,
    i.e. x^{n+1} = x^n + c_tilde dt u^{n+1/2} / gamma^{n+1/2}."""
    g = lorentz_gamma(u_new)
    out = x + (p.c_tilde * p.dt) * u_new / g
    box = (p.nx * p.dx, p.ny * p.dx, p.nz * p.dx)
    return np.stack([wrap(out[d], box[d]) for d in range(3)])


def moments(x, u, p: Params, w=None):
    """CR mass, momentum and energy densities on the grid from the packet totals
    M_j, P_j = M_j c u_j and E_j = M_j c^2 gamma_j (Sec. 2, after Eq. (10)),
    spread by the kernel W and divided by the cell volume (naive mode: c_tilde in
    place of c, naive_constants).  w: optional packet weights N_j / N (losses), which
    scale every packet total."""
    idx, wts = shape_weights(x, p)
    g = lorentz_gamma(u)
    cp = mode_constants(p)[2]
    m = p.mass * np.ones(u.shape[1], dtype=u.dtype)
    if w is not None:
        m = m * w
    vals = np.concatenate([m[None], m * cp * u, (m * cp * cp * g)[None]])
    d = deposit(idx, wts, vals, p.n_cells) / p.volume
    return d[0], d[1:4], d[4]


def step(x, u, E, B, p: Params):
    """One packet step: gather E, B at x^n, kick u^{n-1/2} -> u^{n+1/2}, deposit
    the exchange at x^n with the same weights, drift to x^{n+1}.
    E, B are (3, n_cells).  Returns (x^{n+1}, u^{n+1/2}, dM (3, n_cells), dE (n_cells))
    where dM, dE are this step's momentum and energy given to the gas per unit volume."""
    idx, w = shape_weights(x, p)
    Ep = gather(E, idx, w)
    Bp = gather(B, idx, w)
    h_e, h_b, _, _ = mode_constants(p)
    u_new = kick(u, Ep, Bp, h_e, h_b, p.pusher)
    dP, dEn = exchange(u, u_new, p)
    dep = deposit(idx, w, np.concatenate([dP, dEn[None]]), p.n_cells) / p.volume
    x_new = drift(x, u_new, p)
    return x_new, u_new, dep[0:3], dep[3]


def rollout(x, u, E, B, p: Params, nsteps, keep_history=False):
    """nsteps packet steps from (x^0, u^{-1/2}).  Returns a dict with the final
    state, the last step's exchange, the exchange summed over all steps and,
    on request, the state before every step."""
    dM_sum = np.zeros((3, p.n_cells), dtype=np.result_type(x, u, E, B))
    dE_sum = np.zeros(p.n_cells, dtype=dM_sum.dtype)
    dM = dE = None
    hist = []
    for _ in range(nsteps):
        if keep_history:
            hist.append((x, u))
        x, u, dM, dE = step(x, u, E, B, p)
        dM_sum = dM_sum + dM
        dE_sum = dE_sum + dE
    return dict(x=x, u=u, dM=dM, dE=dE, dM_sum=dM_sum, dE_sum=dE_sum, history=hist)


def coupled_step(x, u, mom, egas, rho, B, p: Params):
    """One packet step coupled to a gas whose density rho and magnetic field B are held
    fixed (no MHD solver).  The gas velocity is u_gas = mom / rho and the step's electric
    field is E = -(u_gas/c) x B with the true c (Sec. 2, after Eq. (5)).  After the packet
    step the gas takes the step's exchange: mom += dM (Eq. (12)) and egas += dE (the same
    rule applied to the packet energy, Eq. (9)).
    rho (n_cells), mom (3, n_cells), egas (n_cells).  Returns (x, u, mom, egas)."""
    E = electric_field(mom / rho, B, p.c)
    x1, u1, dM, dE = step(x, u, E, B, p)
    return x1, u1, mom + dM, egas + dE


def coupled_rollout(x, u, mom, egas, rho, B, p: Params, nsteps):
    """nsteps coupled steps.  Returns the final packets and gas state and the electric
    field of the final gas state (the field the next step would gather)."""
    for _ in range(nsteps):
        x, u, mom, egas = coupled_step(x, u, mom, egas, rho, B, p)
    return dict(x=x, u=u, mom=mom, egas=egas, E=electric_field(mom / rho, B, p.c))


def conserved_totals(u, mom, egas, p: Params, w=None):
    """Totals the CR-gas exchange conserves (Sec. 2, discussion after Eq. (12)): the
    momentum V sum_i (rho u)_i + (c/c_tilde) sum_j P_j with P_j = M_j c u_j, and the
    energy V sum_i e_i + (c/c_tilde) sum_j M_j c^2 gamma_j.  Naive mode: the totals its
    own exchange conserves, with M_j c_tilde u_j, M_j c_tilde^2 gamma_j and no c/c_tilde.
    w: optional packet weights (losses).  Returns (momentum (3,), energy)."""
    _, _, cp, k = mode_constants(p)
    wt = np.ones(u.shape[1]) if w is None else w
    P = p.volume * mom.sum(axis=1) + k * p.mass * cp * (wt * u).sum(axis=1)
    En = p.volume * egas.sum() + k * p.mass * cp * cp * (wt * lorentz_gamma(u)).sum()
    return P, En
