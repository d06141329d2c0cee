"""Seeded synthetic inputs shared by the oracle, the tests and the bench.

This package holds input generation only: hexahedral meshes (connectivity
plus the face/cell geometry a mesh reader would deliver), boundary-condition
tables, initial macroparameter fields and the named workload configurations.
It contains none of the kinetic method's arithmetic (no moments, equilibria,
fluxes or tensor algebra), so both the HIP path and the CPU oracle can take
their inputs from it without sharing any of the computation under test.
"""

from .meshes import (  # noqa: F401
    BC_SYM, BC_INFLOW, BC_OUTFLOW, BC_WALL,
    periodic_box, channel_with_obstacle, jittered_box, merge_meshes,
    check_closed,
)
from .configs import CONFIGS, make_config, initial_macros  # noqa: F401
