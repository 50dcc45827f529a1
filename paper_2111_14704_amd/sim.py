"""A packet simulation on one GPU: device tensors for the grid fields and the
packet state, wired to one librsol handle.  Marshalling only; all arithmetic
runs in librsol."""

from __future__ import annotations

import numpy as np
import torch

from .rsol import RSOL_CIC, RSOL_FP32, RSOL_FP64, RSOL_TSC, Handle, Params


class Simulation:
    """Holds B, u_gas, E ([3, n_cells] float64) and the packet arrays on ``device``.

    ``B``, ``u_gas``: (3, nz, ny, nx) or (3, n_cells) arrays; ``x``, ``u``: (3, Np)
    absolute positions and momenta gamma*beta; ``ids``: (Np,) int32.  ``dt=None``
    takes the RSOL Courant timestep computed by the library.
    """

    def __init__(self, *, n, dx, shape, c, c_tilde, qomc, courant, mass, B, u_gas, x, u, ids,
                 precision="fp64", sort_every=4, flags=0, dt=None, device="cuda"):
        self.device = torch.device(device)
        nx, ny, nz = n
        self.fp32 = precision == "fp32"
        self.params = Params(nx=nx, ny=ny, nz=nz, shape=RSOL_CIC if shape == "cic" else RSOL_TSC,
                             precision=RSOL_FP32 if self.fp32 else RSOL_FP64, dx=dx, c=c, c_tilde=c_tilde,
                             qomc=qomc, dt=0.0, courant=courant, mass=mass, sort_every=sort_every, flags=flags)
        np_ = int(np.asarray(x).shape[1])
        self.n_particles = np_
        self.n_cells = nx * ny * nz
        self.handle = Handle(self.params, np_, device=self.device)
        h = self.handle
        f64 = dict(dtype=torch.float64, device=self.device)
        self.B = torch.as_tensor(np.ascontiguousarray(np.asarray(B).reshape(3, -1)), **f64)
        self.u_gas = torch.as_tensor(np.ascontiguousarray(np.asarray(u_gas).reshape(3, -1)), **f64)
        self.E = torch.empty_like(self.B)
        h.rsol_electric_field(self.u_gas, self.B, self.E)
        h.rsol_set_fields(self.E, self.B)
        self.ids = torch.as_tensor(np.ascontiguousarray(ids, dtype=np.int32), device=self.device)
        x64 = torch.as_tensor(np.ascontiguousarray(x), **f64)
        if self.fp32:
            self.cell = torch.empty(np_, dtype=torch.int32, device=self.device)
            self.off = torch.empty((3, np_), dtype=torch.float32, device=self.device)
            if np_:
                h.rsol_positions_to_cells(x64, self.cell, self.off)
            self.u = torch.as_tensor(np.ascontiguousarray(u), dtype=torch.float32, device=self.device)
            h.rsol_set_particles(self.cell, self.off, self.u, self.ids)
            self.x = None
        else:
            self.x = x64
            self.u = torch.as_tensor(np.ascontiguousarray(u), **f64)
            h.rsol_set_particles(self.x, None, self.u, self.ids)
        if dt is None:
            self.dt = h.rsol_get_dt()  # the handle's dt is unset: it adopts the Courant timestep
        else:
            self.dt = float(dt)
            h.rsol_set_dt(self.dt)

    @classmethod
    def from_workload(cls, w, **kw):
        args = dict(n=(w.nx, w.ny, w.nz), dx=w.dx, shape=w.shape, c=w.c, c_tilde=w.c_tilde, qomc=w.qomc,
                    courant=w.courant, mass=w.mass, B=w.B, u_gas=w.u_gas, x=w.x, u=w.u, ids=w.ids,
                    precision=w.precision)
        args.update(kw)
        return cls(**args)

    def zeros_grid(self, comps):
        return torch.zeros((comps, self.n_cells), dtype=torch.float64, device=self.device)

    def step(self, nsteps, dM=None, dE=None):
        self.handle.rsol_step(nsteps, dM, dE)

    def set_losses(self, sigma, nn, w):
        """Catastrophic losses (needs flags with RSOL_FLAG_LOSSES at construction): nn is the
        nucleon density per cell (n_cells,), w the initial packet weights (Np,); the weights
        live in ``self.w`` (packet precision) and follow the packets."""
        f64 = dict(dtype=torch.float64, device=self.device)
        self.nn = torch.as_tensor(np.ascontiguousarray(np.asarray(nn).reshape(-1)), **f64)
        self.w = torch.as_tensor(np.ascontiguousarray(w), dtype=torch.float32 if self.fp32 else torch.float64,
                                 device=self.device)
        self.handle.rsol_set_losses(sigma, self.nn, self.w)

    def set_weights(self, w):
        """Per-packet weights w_j (Np,) multiplying the packet mass (needs flags with
        RSOL_FLAG_WEIGHTS at construction); they live in ``self.w`` (packet precision) and
        follow the packets."""
        self.w = torch.as_tensor(np.ascontiguousarray(w), dtype=torch.float32 if self.fp32 else torch.float64,
                                 device=self.device)
        self.handle.rsol_set_weights(self.w)

    def sync(self):
        """Bring the registered packet tensors up to date (with RSOL_FLAG_RESIDENT the
        packets stay in the library's cell lists between steps)."""
        self.handle.rsol_sync_particles()

    def weights_by_id(self):
        """Packet weights (float64 numpy) indexed by packet id."""
        self.sync()
        ids = self.ids.cpu().numpy()
        return self.w.double().cpu().numpy()[np.argsort(ids, kind="stable")]

    def step_coupled(self, nsteps, rho, mom, egas=None):
        """nsteps steps coupled to the gas (rho, mom = rho u, egas: float64 device tensors of
        shapes (n_cells,), (3, n_cells), (n_cells,)); mom and egas are updated in place and
        ``self.E`` holds the field of the final gas state."""
        self.handle.rsol_step_coupled(nsteps, rho, mom, egas, self.E)

    def positions64(self):
        """Absolute FP64 positions (3, Np) on the device, in the current packet order."""
        self.sync()
        if not self.fp32:
            return self.x
        x = torch.empty((3, self.n_particles), dtype=torch.float64, device=self.device)
        if self.n_particles:
            self.handle.rsol_cells_to_positions(self.cell, self.off, x)
        return x

    def state_by_id(self):
        """(x, u) as float64 numpy arrays indexed by packet id."""
        self.sync()
        x = self.positions64().cpu().numpy()
        u = self.u.double().cpu().numpy()
        ids = self.ids.cpu().numpy()
        order = np.argsort(ids, kind="stable")
        return x[:, order], u[:, order]

    def moments(self):
        rho = self.zeros_grid(1)[0]
        P = self.zeros_grid(3)
        e = self.zeros_grid(1)[0]
        self.handle.rsol_moments(rho, P, e)
        return rho, P, e
