"""Seeded synthetic inputs for the RSOL MHD-PIC hot path.

This package only draws random numbers and lays them out in arrays: grid
fields of a prescribed MHD background (magnetic field B and gas velocity u),
cosmic-ray packet positions and momenta, and the run parameters. It performs
none of the method's arithmetic (no electric field, no interpolation, no push,
no deposit, no timestep rule); both the CPU oracle and the GPU path take these
arrays as their common input.
"""

from .configs import Workload, make_workload, gas_state, loss_state, WORKLOADS, UNITS  # noqa: F401
