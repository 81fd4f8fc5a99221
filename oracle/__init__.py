"""CPU oracle of the oscillating-body lattice-BGK method.

TEST INFRASTRUCTURE ONLY.  Imported by tests, by the smoke check and by the
benchmark's CPU-baseline leg; the product library never imports it.
"""
from .oracle import (  # noqa: F401
    GEOM_BOX, GEOM_PERIODIC, GEOM_PLATE, FAR_EQ, FAR_WALL, COLL_BGK, COLL_REGULARIZED, WALL_BB, WALL_DS,
    WALL_MAXWELL,
    OracleParams, advect, collide, equilibrium, lattice, lockin_fit, run,
)
