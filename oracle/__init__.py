"""Plain FP64 CPU oracle of the cRKDG hot path.  Test infrastructure only:
imported by the test suite, the smoke check and the benchmark's CPU-baseline
leg, never by the library."""
from .crkdg_oracle import (ADVECTION, BURGERS, EULER, SHALLOW_WATER, PERIODIC, OUTFLOW, REFLECT, DIRICHLET,  # noqa: F401
                           BUTCHER,
                           CRKDG, Problem, gauss_legendre, gauss_lobatto, legendre_table,
                           lagrange_1d, make)
