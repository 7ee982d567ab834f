"""Seeded synthetic initial fields shared by the reference and the GPU path.

This package only samples velocity / pressure fields at cell centres.  It holds
none of the lattice Boltzmann arithmetic (no equilibria, no moments, no
streaming): both sides receive the arrays produced here as plain FP64 inputs.
"""

from .fields import (  # noqa: F401
    cell_centres,
    taylor_green,
    taylor_green_pressure,
    shear_wave,
    abc_flow,
    abc_pressure,
    random_field_2d,
    random_field_3d,
    random_field_box,
    random_pressure_2d,
    pressure_coefficients,
    pressure_at,
    well_prepared_density,
    batch_run_specs,
)
