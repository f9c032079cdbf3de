"""Seeded synthetic inputs shared by the tests, the CPU oracle checks and the benchmark.

Only input construction lives here: random SU(3) gauge links, unit and pure-gauge
links, gauge transformations of a link field, random spinor fields and plane waves.
None of the trace-estimation arithmetic (operator, solvers, projections, estimator)
is here; both the HIP library and the oracle take what this package returns.
"""
from .fields import (  # noqa: F401
    GELL_MANN,
    gauge_transform,
    lattice_volume,
    pure_gauge_links,
    random_su3,
    random_spinors,
    su3_links,
    unit_links,
    plane_wave,
    transform_spinor,
)
