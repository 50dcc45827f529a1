"""The five seeded synthetic workloads of the RSOL MHD-PIC hot path.

Unit system (the paper fixes none, see Sec. 2): cell size dx = 1 (V = 1), gas
density rho = 1, mean field B0 = 1, Alfven speed v_A = B0/sqrt(rho) = 1, true
speed of light c = 1000 v_A, and q/(m c) = 4 c, so that a packet with
u_perp = gamma*beta_perp = 1 gyrates with radius 0.25 dx in B0 on the grid.

Each workload is generated from ``numpy.random.SeedSequence(seed).spawn(5)``,
one stream each for [positions, directions, momentum magnitudes, field modes,
loss target and gradient-check coordinates]; ``gas_state`` draws from a sixth
child of the same seed sequence.  Positions are stratified: exactly
``ppc`` packets per cell, packet j = cell * ppc + k with
cell = ix + nx * (iy + ny * iz), offsets uniform in the cell.

Only random draws and array layout live here; the electric field, the
timestep, the push and every deposit belong to the method and are computed by
the oracle and by the GPU library separately.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

UNITS = dict(dx=1.0, rho=1.0, B0=1.0, c=1000.0, qomc=4000.0, courant=0.3)


@dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    ppc: int
    shape: str              # "cic" or "tsc"
    c: float
    c_tilde: float
    qomc: float
    courant: float
    dx: float
    nsteps: int
    precision: str          # "fp64" or "fp32"
    mass: float             # uniform packet mass weight M_j = N_j m_s
    B: np.ndarray           # (3, nz, ny, nx) cell-centred magnetic field
    u_gas: np.ndarray       # (3, nz, ny, nx) cell-centred gas velocity
    x: np.ndarray           # (3, Np) absolute packet positions in [0, L)
    u: np.ndarray           # (3, Np) packet momenta gamma*beta at t = -dt/2
    ids: np.ndarray         # (Np,) int32 packet labels
    ckpt_every: int = 0
    target: Optional[np.ndarray] = None      # (3, nz, ny, nx) loss target
    grad_coords: list = field(default_factory=list)

    @property
    def n_cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_particles(self) -> int:
        return self.x.shape[1]

    @property
    def box(self):
        return (self.nx * self.dx, self.ny * self.dx, self.nz * self.dx)


def _stratified_positions(rng, nx, ny, nz, ppc, dx):
    n_cells = nx * ny * nz
    cell = np.repeat(np.arange(n_cells, dtype=np.int64), ppc)
    ix = cell % nx
    iy = (cell // nx) % ny
    iz = cell // (nx * ny)
    off = rng.random((3, cell.size))
    x = np.empty((3, cell.size))
    x[0] = (ix + off[0]) * dx
    x[1] = (iy + off[1]) * dx
    x[2] = (iz + off[2]) * dx
    # an offset that rounds up to the cell edge is moved to the same cell's start
    for d, n in enumerate((nx, ny, nz)):
        np.copyto(x[d], 0.0, where=x[d] >= n * dx)
    return x


def _isotropic_directions(rng, n):
    mu = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * np.pi, n)
    s = np.sqrt(1.0 - mu * mu)
    return np.stack([mu, s * np.cos(phi), s * np.sin(phi)])


def _power_law(rng, n, p1, p2, index=4.5):
    """Magnitudes with dN/dp proportional to p**-index on [p1, p2] (inverse CDF)."""
    a = 1.0 - index
    xi = rng.random(n)
    return (p1 ** a + xi * (p2 ** a - p1 ** a)) ** (1.0 / a)


def _alfven_modes_along_x(rng, nx, ny, nz, dx, n_modes, rms):
    """Transverse waves with k along x, random phase and polarisation angle."""
    phase = rng.uniform(0.0, 2.0 * np.pi, n_modes)
    psi = rng.uniform(0.0, 2.0 * np.pi, n_modes)
    amp = rms * np.sqrt(2.0 / n_modes)
    xc = (np.arange(nx) + 0.5) * dx
    L = nx * dx
    dB = np.zeros((3, nz, ny, nx))
    for m in range(n_modes):
        k = 2.0 * np.pi * (m + 1) / L
        prof = amp * np.cos(k * xc + phase[m])
        dB[1] += np.cos(psi[m]) * prof[None, None, :]
        dB[2] += np.sin(psi[m]) * prof[None, None, :]
    return dB


def _alfvenic_turbulence(rng, nx, ny, nz, b0, n_max, rms):
    """Isotropic random-phase field, |dB_k| ~ |k|^(-11/6) (shell spectrum k^-5/3),
    polarised along k x b0 (perpendicular to k and to the mean field)."""
    kz = np.fft.fftfreq(nz) * nz
    ky = np.fft.fftfreq(ny) * ny
    kx = np.fft.rfftfreq(nx) * nx
    KZ, KY, KX = np.meshgrid(kz, ky, kx, indexing="ij")
    kmag = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    live = (kmag >= 1.0) & (kmag <= n_max)
    amp = np.zeros_like(kmag)
    amp[live] = kmag[live] ** (-11.0 / 6.0)
    # polarisation e = k x b0 / |k x b0|; k parallel to b0 takes z-hat (perpendicular to both)
    ex = KY * b0[2] - KZ * b0[1]
    ey = KZ * b0[0] - KX * b0[2]
    ez = KX * b0[1] - KY * b0[0]
    en = np.sqrt(ex ** 2 + ey ** 2 + ez ** 2)
    par = en < 1e-12
    en[par] = 1.0
    ex, ey, ez = ex / en, ey / en, ez / en
    ex[par], ey[par], ez[par] = 0.0, 0.0, 1.0
    phase = rng.uniform(0.0, 2.0 * np.pi, kmag.shape)
    spec = amp * np.exp(1j * phase)
    dB = np.stack([np.fft.irfftn(spec * e, s=(nz, ny, nx), axes=(0, 1, 2)) for e in (ex, ey, ez)])
    scale = rms / np.sqrt(np.mean(np.sum(dB * dB, axis=0)))
    return dB * scale


def _equipartition_mass(u, n_cells, dx, B0, c):
    """Uniform packet mass weight making the initial mean CR energy density equal
    to the magnetic energy density B0^2/2 (total CR energy / (c^2 sum gamma))."""
    gamma_sum = np.sum(np.sqrt(1.0 + np.sum(u * u, axis=0)))
    return 0.5 * B0 * B0 * n_cells * dx ** 3 / (c * c * gamma_sum)


# name, grid, ppc, shape, c/c_tilde, steps, precision
WORKLOADS = {
    1: dict(name="uniform-16c-8ppc-cic-fp64", n=16, ppc=8, shape="cic", ratio=10.0, nsteps=100, precision="fp64"),
    2: dict(name="alfven-64c-64ppc-tsc-fp64", n=64, ppc=64, shape="tsc", ratio=30.0, nsteps=200, precision="fp64"),
    3: dict(name="uniform-16c-8ppc-cic-fp32", n=16, ppc=8, shape="cic", ratio=10.0, nsteps=100, precision="fp32"),
    4: dict(name="turb-128c-32ppc-tsc-fp32", n=128, ppc=32, shape="tsc", ratio=100.0, nsteps=100, precision="fp32"),
    5: dict(name="grad-32c-32ppc-cic", n=32, ppc=32, shape="cic", ratio=10.0, nsteps=256, precision="fp64"),
}


def make_workload(k: int, seed: int = 0, n: Optional[int] = None, ppc: Optional[int] = None,
                  nsteps: Optional[int] = None, ratio: Optional[float] = None,
                  precision: Optional[str] = None) -> Workload:
    """Build workload ``k`` (1..5).  ``n``, ``ppc``, ``nsteps``, ``ratio`` (= c/c_tilde)
    and ``precision`` override the defaults to make smaller variants of the same recipe."""
    spec = dict(WORKLOADS[k])
    n = spec["n"] if n is None else n
    ppc = spec["ppc"] if ppc is None else ppc
    nsteps = spec["nsteps"] if nsteps is None else nsteps
    ratio = spec["ratio"] if ratio is None else ratio
    precision = spec["precision"] if precision is None else precision
    nx = ny = nz = n
    dx, B0, c, qomc = UNITS["dx"], UNITS["B0"], UNITS["c"], UNITS["qomc"]
    s_pos, s_dir, s_mag, s_fld, s_aux = np.random.SeedSequence(seed).spawn(5)
    r_pos, r_dir, r_mag, r_fld, r_aux = (np.random.default_rng(s) for s in (s_pos, s_dir, s_mag, s_fld, s_aux))

    x = _stratified_positions(r_pos, nx, ny, nz, ppc, dx)
    npart = x.shape[1]
    dirs = _isotropic_directions(r_dir, npart)

    B = np.zeros((3, nz, ny, nx))
    u_gas = np.zeros((3, nz, ny, nx))
    if k in (1, 3, 5):
        B[0] = B0
        u = 10.0 * dirs
    elif k == 2:
        B[0] = B0
        dB = _alfven_modes_along_x(r_fld, nx, ny, nz, dx, 32, 1e-2 * B0)
        B += dB
        u_gas = -dB / np.sqrt(UNITS["rho"])
        u = _power_law(r_mag, npart, 1.0, 100.0) * dirs
        # bulk drift of 5 v_A along x: Lorentz boost of each packet's 4-momentum
        beta_d = 5.0 / c
        gamma_d = 1.0 / np.sqrt(1.0 - beta_d * beta_d)
        g = np.sqrt(1.0 + np.sum(u * u, axis=0))
        u[0] = gamma_d * (u[0] + beta_d * g)
    elif k == 4:
        b0 = np.array([1.0, 1.0, 0.0]) / np.sqrt(2.0)
        dB = _alfvenic_turbulence(r_fld, nx, ny, nz, b0, 32, 0.1 * B0)
        B = b0[:, None, None, None] * B0 + dB
        u_gas = -dB / np.sqrt(UNITS["rho"])
        u = _power_law(r_mag, npart, 1.0, 1000.0) * dirs
    else:
        raise ValueError(f"unknown workload {k}")

    mass = _equipartition_mass(u, nx * ny * nz, dx, B0, c)
    w = Workload(name=spec["name"], nx=nx, ny=ny, nz=nz, ppc=ppc, shape=spec["shape"], c=c,
                 c_tilde=c / ratio, qomc=qomc, courant=UNITS["courant"], dx=dx, nsteps=nsteps,
                 precision=precision, mass=mass, B=B, u_gas=u_gas, x=x, u=u,
                 ids=np.arange(npart, dtype=np.int32))
    if k == 5:
        w.ckpt_every = 16
        # seeded target: per-component rms of an isotropic cell's momentum density
        sigma = mass * c * 10.0 * np.sqrt(ppc / 3.0) / dx ** 3
        w.target = sigma * r_aux.standard_normal((3, nz, ny, nx))
        nc = nx * ny * nz
        coords = []
        for kind, cnt, hi in (("E", 16, nc), ("B", 16, nc), ("u", 32, npart)):
            comp = r_aux.integers(0, 3, cnt)
            where = r_aux.integers(0, hi, cnt)
            coords += [(kind, int(a), int(b)) for a, b in zip(comp, where)]
        w.grad_coords = coords
    return w


def gas_state(w: Workload, seed: int = 0):
    """Seeded gas for runs coupled to the packets (density and B held fixed): density
    rho = UNITS["rho"] * U(0.5, 1.5) per cell, momentum density rho * u_gas, and an energy
    density U(1, 2) times the mean magnetic energy density B0^2/2.
    Returns (rho (n_cells,), mom (3, n_cells), egas (n_cells,)) as float64."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(6)[5])
    nc = w.n_cells
    rho = UNITS["rho"] * rng.uniform(0.5, 1.5, nc)
    mom = rho * w.u_gas.reshape(3, -1)
    egas = 0.5 * UNITS["B0"] ** 2 * rng.uniform(1.0, 2.0, nc)
    return rho, np.ascontiguousarray(mom), egas


def loss_state(w: Workload, seed: int = 0):
    """Nucleon density and loss cross-section for runs with catastrophic losses: n_n is
    the gas density of ``gas_state`` (nucleon mass 1 in code units) and sigma is set so
    that the mean free path 1/(sigma <n_n>) is 40 cells.  Packets start with weight 1.
    Returns (nn (n_cells,), sigma, weights (Np,))."""
    rho, _, _ = gas_state(w, seed)
    nn = rho / 1.0
    sigma = 1.0 / (40.0 * w.dx * float(nn.mean()))
    return nn, sigma, np.ones(w.n_particles)
