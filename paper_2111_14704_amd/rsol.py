"""ctypes binding of librsol (include/rsol.h).

Argument marshalling only: every function forwards to the C entry point of the
same name with device pointers taken from torch tensors; all arithmetic of the
method runs in the library's HIP kernels.  Loading fails loudly when the
library has not been built (python -m paper_2111_14704_amd.build).
"""

from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librsol.so")

RSOL_OK = 0
STATUS = {
    -1: "RSOL_EINVAL", -2: "RSOL_ESTATE", -3: "RSOL_EHIP", -4: "RSOL_ECOURANT",
    -5: "RSOL_ENAN", -6: "RSOL_ESCRATCH", -7: "RSOL_ETILE",
}
RSOL_CIC, RSOL_TSC = 1, 2
RSOL_FP64, RSOL_FP32 = 0, 1
RSOL_FLAG_KEEP_ORDER = 1
RSOL_FLAG_TILED = 2
RSOL_FLAG_NAIVE = 4
RSOL_FLAG_LOSSES = 8
RSOL_FLAG_WEIGHTS = 8
RSOL_FLAG_PUSHER_VAY = 16
RSOL_FLAG_PUSHER_HC = 32
RSOL_FLAG_RESIDENT = 64
RSOL_FLAG_RECORD_ONLY = 128


class RSOLError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


class rsol_params(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("shape", ctypes.c_int32), ("precision", ctypes.c_int32), ("sort_every", ctypes.c_int32),
        ("flags", ctypes.c_int32), ("reserved", ctypes.c_int32),
        ("dx", ctypes.c_double), ("c", ctypes.c_double), ("c_tilde", ctypes.c_double),
        ("qomc", ctypes.c_double), ("dt", ctypes.c_double), ("courant", ctypes.c_double),
        ("mass", ctypes.c_double),
    ]


_lib = None


def lib():
    """The loaded librsol.so (raises if it is missing)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2111_14704_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        P = ctypes.POINTER(rsol_params)
        sig = {
            "rsol_scratch_bytes": (ctypes.c_size_t, [P, i64]),
            "rsol_init": (ctypes.c_int, [P, i64, vp, vp, ctypes.c_size_t, ctypes.POINTER(vp)]),
            "rsol_destroy": (ctypes.c_int, [vp]),
            "rsol_last_error": (ctypes.c_char_p, [vp]),
            "rsol_electric_field": (ctypes.c_int, [vp, vp, vp, vp]),
            "rsol_set_fields": (ctypes.c_int, [vp, vp, vp]),
            "rsol_set_particles": (ctypes.c_int, [vp, vp, vp, vp, vp]),
            "rsol_positions_to_cells": (ctypes.c_int, [vp, vp, vp, vp]),
            "rsol_cells_to_positions": (ctypes.c_int, [vp, vp, vp, vp]),
            "rsol_courant_dt": (ctypes.c_int, [vp, ctypes.POINTER(dbl)]),
            "rsol_set_dt": (ctypes.c_int, [vp, dbl]),
            "rsol_get_dt": (ctypes.c_int, [vp, ctypes.POINTER(dbl)]),
            "rsol_gather": (ctypes.c_int, [vp, vp, vp]),
            "rsol_push": (ctypes.c_int, [vp, vp, vp, vp]),
            "rsol_deposit": (ctypes.c_int, [vp, vp, vp, vp]),
            "rsol_drift": (ctypes.c_int, [vp]),
            "rsol_sort": (ctypes.c_int, [vp]),
            "rsol_step": (ctypes.c_int, [vp, i32, vp, vp]),
            "rsol_step_coupled": (ctypes.c_int, [vp, i32, vp, vp, vp, vp]),
            "rsol_set_losses": (ctypes.c_int, [vp, dbl, vp, vp]),
            "rsol_set_weights": (ctypes.c_int, [vp, vp]),
            "rsol_moments": (ctypes.c_int, [vp, vp, vp, vp]),
            "rsol_sync_particles": (ctypes.c_int, [vp]),
            "rsol_check": (ctypes.c_int, [vp]),
            "rsol_timing": (ctypes.c_int, [vp, i32]),
            "rsol_stray_count": (ctypes.c_int, [vp, ctypes.POINTER(i64)]),
            "rsol_set_flags": (ctypes.c_int, [vp, i32]),
            "rsol_state_bytes": (ctypes.c_size_t, [vp]),
            "rsol_record_states": (ctypes.c_int, [vp, i32, vp]),
            "rsol_step_backward": (ctypes.c_int, [vp, i32, vp, vp, vp, vp, vp, vp, vp]),
            "rsol_moments_backward": (ctypes.c_int, [vp, vp, vp, vp, vp, vp]),
            "rsol_timing_read": (ctypes.c_int, [vp, ctypes.POINTER(dbl), ctypes.POINTER(i64),
                                                 ctypes.POINTER(dbl), ctypes.POINTER(i64)]),
            "rsol_step_static": (ctypes.c_int, [P, i64, vp, vp, vp, vp, vp, vp, vp, i32, vp, vp]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return [
        "rsol_scratch_bytes", "rsol_init", "rsol_destroy", "rsol_last_error", "rsol_electric_field",
        "rsol_set_fields", "rsol_set_particles", "rsol_positions_to_cells", "rsol_cells_to_positions",
        "rsol_courant_dt", "rsol_set_dt", "rsol_get_dt", "rsol_gather", "rsol_push", "rsol_deposit", "rsol_drift",
        "rsol_sort", "rsol_step", "rsol_moments", "rsol_check", "rsol_timing", "rsol_timing_read",
        "rsol_stray_count", "rsol_set_flags", "rsol_state_bytes", "rsol_record_states", "rsol_step_backward",
        "rsol_moments_backward", "rsol_step_coupled", "rsol_set_losses", "rsol_sync_particles",
        "rsol_step_static", "rsol_set_weights",
    ]


def _ptr(t):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("librsol takes device tensors")
    if not t.is_contiguous():
        raise ValueError("librsol takes contiguous tensors")
    return ctypes.c_void_p(t.data_ptr())


def _check(h, rc):
    if rc != RSOL_OK:
        msg = lib().rsol_last_error(h)
        raise RSOLError(rc, msg.decode() if msg else "")


@dataclass
class Params:
    nx: int
    ny: int
    nz: int
    shape: int
    precision: int
    dx: float
    c: float
    c_tilde: float
    qomc: float
    dt: float = 0.0
    courant: float = 0.3
    mass: float = 1.0
    sort_every: int = 4
    flags: int = 0

    def to_c(self) -> rsol_params:
        return rsol_params(self.nx, self.ny, self.nz, self.shape, self.precision, self.sort_every, self.flags, 0,
                           self.dx, self.c, self.c_tilde, self.qomc, self.dt, self.courant, self.mass)


def rsol_scratch_bytes(params: Params, n_particles: int) -> int:
    p = params.to_c()
    n = lib().rsol_scratch_bytes(ctypes.byref(p), n_particles)
    if n == 0:
        raise RSOLError(-1, "invalid parameters")
    return n


def rsol_step_static(params: Params, pos, off, u, ids, E, B, nsteps: int, dM=None, dE=None, stream=None):
    """rsol_step_static: nsteps steps of the packets (pos, off, u, ids: device tensors of
    the precision's layout, updated in place) in the fields E, B with params.dt, using the
    library's static device scratch (no device allocation, no handle)."""
    n = int(u.shape[1])
    p = params.to_c()
    st = stream if stream is not None else torch.cuda.current_stream(u.device)
    rc = lib().rsol_step_static(ctypes.byref(p), n, ctypes.c_void_p(st.cuda_stream), _ptr(E), _ptr(B), _ptr(pos),
                                _ptr(off), _ptr(u), _ptr(ids), int(nsteps), _ptr(dM), _ptr(dE))
    if rc != RSOL_OK:
        msg = lib().rsol_last_error(None)
        raise RSOLError(rc, msg.decode() if msg else "")


class Handle:
    """An rsol handle plus the caller-owned scratch tensor it uses."""

    def __init__(self, params: Params, n_particles: int, device="cuda", stream=None):
        self.params = params
        self.n = int(n_particles)
        self.device = torch.device(device)
        nbytes = rsol_scratch_bytes(params, self.n)
        # 256-byte aligned (the caching allocator aligns blocks to 512 bytes)
        self.scratch = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        p = params.to_c()
        rc = lib().rsol_init(ctypes.byref(p), self.n, ctypes.c_void_p(self.stream.cuda_stream),
                             _ptr(self.scratch), nbytes, ctypes.byref(h))
        if rc != RSOL_OK:
            raise RSOLError(rc, lib().rsol_last_error(None).decode())
        self.h = h
        self._keep = {}

    def close(self):
        if self.h:
            lib().rsol_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------------ 1:1 entry points
    def rsol_electric_field(self, u_gas, B, E):
        _check(self.h, lib().rsol_electric_field(self.h, _ptr(u_gas), _ptr(B), _ptr(E)))

    def rsol_set_fields(self, E, B):
        self._keep["E"], self._keep["B"] = E, B
        _check(self.h, lib().rsol_set_fields(self.h, _ptr(E), _ptr(B)))

    def rsol_set_losses(self, sigma: float, nn, w):
        self._keep.update(nn=nn, w=w)
        _check(self.h, lib().rsol_set_losses(self.h, float(sigma), _ptr(nn), _ptr(w)))

    def rsol_set_weights(self, w):
        self._keep["w"] = w
        _check(self.h, lib().rsol_set_weights(self.h, _ptr(w)))

    def rsol_set_particles(self, pos, off, u, ids):
        self._keep.update(pos=pos, off=off, u=u, ids=ids)
        _check(self.h, lib().rsol_set_particles(self.h, _ptr(pos), _ptr(off), _ptr(u), _ptr(ids)))

    def rsol_positions_to_cells(self, x, cell, off):
        _check(self.h, lib().rsol_positions_to_cells(self.h, _ptr(x), _ptr(cell), _ptr(off)))

    def rsol_cells_to_positions(self, cell, off, x):
        _check(self.h, lib().rsol_cells_to_positions(self.h, _ptr(cell), _ptr(off), _ptr(x)))

    def rsol_courant_dt(self) -> float:
        dt = ctypes.c_double()
        _check(self.h, lib().rsol_courant_dt(self.h, ctypes.byref(dt)))
        return dt.value

    def rsol_set_dt(self, dt: float):
        _check(self.h, lib().rsol_set_dt(self.h, float(dt)))

    def rsol_get_dt(self) -> float:
        dt = ctypes.c_double()
        _check(self.h, lib().rsol_get_dt(self.h, ctypes.byref(dt)))
        return dt.value

    def rsol_gather(self, Ep, Bp):
        _check(self.h, lib().rsol_gather(self.h, _ptr(Ep), _ptr(Bp)))

    def rsol_push(self, Ep, Bp, payload):
        _check(self.h, lib().rsol_push(self.h, _ptr(Ep), _ptr(Bp), _ptr(payload)))

    def rsol_deposit(self, payload, dM, dE=None):
        _check(self.h, lib().rsol_deposit(self.h, _ptr(payload), _ptr(dM), _ptr(dE)))

    def rsol_drift(self):
        _check(self.h, lib().rsol_drift(self.h))

    def rsol_sort(self):
        _check(self.h, lib().rsol_sort(self.h))

    def rsol_step(self, nsteps: int, dM=None, dE=None):
        _check(self.h, lib().rsol_step(self.h, int(nsteps), _ptr(dM), _ptr(dE)))

    def rsol_step_coupled(self, nsteps: int, rho, mom, egas, E):
        self._keep.update(rho=rho, mom=mom, egas=egas, E=E)
        _check(self.h, lib().rsol_step_coupled(self.h, int(nsteps), _ptr(rho), _ptr(mom), _ptr(egas), _ptr(E)))

    def rsol_sync_particles(self):
        _check(self.h, lib().rsol_sync_particles(self.h))

    def rsol_moments(self, rho=None, P=None, e=None):
        _check(self.h, lib().rsol_moments(self.h, _ptr(rho), _ptr(P), _ptr(e)))

    def rsol_check(self):
        _check(self.h, lib().rsol_check(self.h))

    def rsol_set_flags(self, flags: int):
        _check(self.h, lib().rsol_set_flags(self.h, int(flags)))
        self.params.flags = int(flags)

    def rsol_state_bytes(self) -> int:
        return int(lib().rsol_state_bytes(self.h))

    def rsol_record_states(self, nsteps: int, states):
        _check(self.h, lib().rsol_record_states(self.h, int(nsteps), _ptr(states)))

    def rsol_step_backward(self, nsteps: int, states, lam_x, lam_u, gE, gB, lam_dM=None, lam_dE=None):
        _check(self.h, lib().rsol_step_backward(self.h, int(nsteps), _ptr(states), _ptr(lam_x), _ptr(lam_u),
                                                _ptr(lam_dM), _ptr(lam_dE), _ptr(gE), _ptr(gB)))

    def rsol_moments_backward(self, lam_x, lam_u, lam_rho=None, lam_P=None, lam_e=None):
        _check(self.h, lib().rsol_moments_backward(self.h, _ptr(lam_rho), _ptr(lam_P), _ptr(lam_e), _ptr(lam_x),
                                                   _ptr(lam_u)))

    def rsol_stray_count(self) -> int:
        n = ctypes.c_int64()
        _check(self.h, lib().rsol_stray_count(self.h, ctypes.byref(n)))
        return n.value

    def rsol_timing(self, enable: bool):
        _check(self.h, lib().rsol_timing(self.h, 1 if enable else 0))

    def rsol_timing_read(self):
        """(step_ms, n_step, sort_ms, n_sort) summed since the last read."""
        a, b = ctypes.c_double(), ctypes.c_int64()
        c, d = ctypes.c_double(), ctypes.c_int64()
        _check(self.h, lib().rsol_timing_read(self.h, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c),
                                              ctypes.byref(d)))
        return a.value, b.value, c.value, d.value
