"""MI355X (gfx950) library for the data-parallel hot path of the reduced-speed-of-light
MHD-PIC method (Ji & Hopkins, arXiv:2111.14704): gather, relativistic Boris push
with the RSOL factors, exchange deposit and drift of cosmic-ray packets.

The compute path is librsol.so (HIP kernels behind the C ABI of include/rsol.h);
this package only binds it (rsol.py) and wires device tensors to it (sim.py).
"""

from .rsol import (  # noqa: F401
    Handle, Params, RSOLError, RSOL_CIC, RSOL_TSC, RSOL_FP32, RSOL_FP64, RSOL_FLAG_KEEP_ORDER, lib,
)
