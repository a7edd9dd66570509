"""CPU oracle for the tDPD + RBC time step (test infrastructure).

Only the tests, the smoke check and the benchmark's CPU-baseline leg import
this package.  It wraps the plain C implementation in tdpd_oracle.c; see that
file's header for the equations it follows and the readings it takes.
"""
from .oracle import Oracle, build_oracle, philox4x32, u01, pair_normals, pair_normals4, pair_normals_batch, TERMS_ALL, TERM  # noqa: F401
