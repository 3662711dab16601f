"""FP64 CPU oracle for the symmetric free-energy multicomponent LB method.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg use this package; the GPU library never does.
"""
from .oracle import Oracle, OracleParams, lattice_tables, feq, forcing, mu_site, psi_site  # noqa: F401
