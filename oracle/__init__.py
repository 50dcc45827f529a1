"""CPU reference oracle for the RSOL MHD-PIC hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path (the HIP library and
its Python binding) may import, call or link this package; only the tests, the
smoke check in ``__graft_entry__`` and the ``cpu_baseline`` leg of ``bench.py``
use it.  It shares no code with the GPU path.

Plain numpy in float64 (complex128 for complex-step derivatives), no tiling,
no sorting, absolute positions.  Every function cites the passage of Ji &
Hopkins, "A Reduced-Speed-of-Light Formulation of the MHD-PIC Method"
(arXiv:2111.14704) that it follows.  Equation numbers count the paper's
displayed equations in order: (1) Lorentz force, (3) RSOL Vlasov equation,
(4) packet decomposition, (5) packet momentum equation, (6)-(10) definitions
of v_eff, beta, gamma, E, p, (11) momentum equation in terms of gamma*beta,
(12) back-reaction on the gas.  ``coupled_step`` closes the gas side of Eq. (12)
with a held-fixed density and magnetic field.
"""

from .pic import (  # noqa: F401
    Params, electric_field, courant_dt, shape_weights, gather, deposit, boris_kick,
    exchange, drift, wrap, moments, step, rollout, lorentz_gamma, coupled_step, coupled_rollout,
    conserved_totals, naive_constants, rsol_constants, mode_constants, loss_factor, exchange_weighted,
    step_with_losses, rollout_with_losses, vay_kick, hc_kick, kick,
)
