"""Host-side checks of the C ABI that need no GPU: the library loads, exports every
entry point include/rsol.h declares, sizes scratch, and rejects bad arguments before
touching the device."""

import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rsol.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rsol_[a-z_0-9]+)\s*\(", text)))


def _lib():
    from paper_2111_14704_amd import rsol
    return rsol, rsol.lib()


def test_header_declares_the_hot_path_entry_points():
    names = _declared()
    for required in ("rsol_init", "rsol_gather", "rsol_push", "rsol_deposit", "rsol_step", "rsol_step_backward"):
        assert required in names, required


def test_library_exports_every_declared_symbol():
    rsol, L = _lib()
    for name in _declared():
        assert hasattr(L, name), name
        getattr(L, name)  # resolves the symbol


def _params(rsol, **kw):
    p = rsol.Params(nx=16, ny=16, nz=16, shape=rsol.RSOL_TSC, precision=rsol.RSOL_FP64, dx=1.0, c=1000.0,
                    c_tilde=100.0, qomc=4000.0, dt=0.0, courant=0.3, mass=1.0, sort_every=4)
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_scratch_bytes_positive_and_grows_with_packets():
    rsol, L = _lib()
    a = rsol.rsol_scratch_bytes(_params(rsol), 1000)
    b = rsol.rsol_scratch_bytes(_params(rsol), 100000)
    c = rsol.rsol_scratch_bytes(_params(rsol, precision=rsol.RSOL_FP32), 100000)
    assert 0 < a < b and 0 < c < b


@pytest.mark.parametrize("bad", [
    dict(nx=0), dict(nx=2000), dict(shape=3), dict(precision=2), dict(sort_every=0), dict(sort_every=9),
    dict(dx=0.0), dict(c_tilde=2000.0), dict(c_tilde=0.0), dict(courant=0.0), dict(courant=0.9),
    dict(mass=-1.0), dict(dt=float("nan")),
    dict(flags=256), dict(flags=16 | 32), dict(flags=2 | 16), dict(flags=2 | 32),
])
def test_invalid_parameters_are_rejected_before_any_device_work(bad):
    rsol, L = _lib()
    p = _params(rsol, **bad).to_c()
    assert L.rsol_scratch_bytes(ctypes.byref(p), 100) == 0
    h = ctypes.c_void_p()
    # a bogus but aligned scratch address: validation must fail before it is used
    rc = L.rsol_init(ctypes.byref(p), 100, None, ctypes.c_void_p(4096), 1 << 40, ctypes.byref(h))
    assert rc == -1
    assert h.value is None
    assert L.rsol_last_error(None)


def test_loss_layout_needs_more_scratch_and_pushers_do_not():
    """RSOL_FLAG_LOSSES sizes the cell-list slot stores for packet weights; the pusher and
    naive flags change only constants (same layout)."""
    rsol, L = _lib()
    base = rsol.rsol_scratch_bytes(_params(rsol), 100000)
    assert rsol.rsol_scratch_bytes(_params(rsol, flags=8), 100000) > base
    for fl in (4, 16, 32, 1 | 16):
        assert rsol.rsol_scratch_bytes(_params(rsol, flags=fl), 100000) == base


def test_small_or_misaligned_scratch_is_rejected():
    rsol, L = _lib()
    p = _params(rsol).to_c()
    need = L.rsol_scratch_bytes(ctypes.byref(p), 100)
    h = ctypes.c_void_p()
    assert L.rsol_init(ctypes.byref(p), 100, None, ctypes.c_void_p(4096), need - 1, ctypes.byref(h)) == -6
    assert L.rsol_init(ctypes.byref(p), 100, None, ctypes.c_void_p(4097), need, ctypes.byref(h)) == -1
    assert L.rsol_init(ctypes.byref(p), 100, None, None, need, ctypes.byref(h)) == -1


def test_null_handle_calls_fail_cleanly():
    rsol, L = _lib()
    assert L.rsol_step(None, 1, None, None) == -1
    assert L.rsol_step_coupled(None, 1, None, None, None, None) == -1
    assert L.rsol_check(None) == -1
    assert L.rsol_sync_particles(None) == -1
    assert L.rsol_moments(None, None, None, None) == -1
    assert L.rsol_set_weights(None, None) == -1
    dt = ctypes.c_double(-1.0)
    assert L.rsol_get_dt(None, ctypes.byref(dt)) == -1 and dt.value == -1.0
    assert L.rsol_destroy(None) == 0


def test_too_many_packets_for_the_cell_lists_are_refused():
    """The default path addresses the id and weight arrays of its slot stores (up to 8
    bytes per slot) with 32-bit byte offsets: a problem whose slot count would take them
    past 4 GiB is refused before any device work."""
    rsol, L = _lib()
    p = _params(rsol, nx=128, ny=128, nz=128).to_c()
    assert L.rsol_scratch_bytes(ctypes.byref(p), 32 * 128 ** 3) > 0
    assert L.rsol_scratch_bytes(ctypes.byref(p), 96 * 128 ** 3) > 0
    assert L.rsol_scratch_bytes(ctypes.byref(p), 128 * 128 ** 3) == 0
    h = ctypes.c_void_p()
    assert L.rsol_init(ctypes.byref(p), 128 * 128 ** 3, None, ctypes.c_void_p(4096), 1 << 40, ctypes.byref(h)) == -1
    assert b"too many packets" in L.rsol_last_error(None)
