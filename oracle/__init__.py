"""FP64 CPU oracle of the coupled ferrofluid compound-droplet step.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the CPU-baseline
leg of the benchmark, never by the product package.  The arithmetic lives in
``fcd_oracle.c`` (plain C, built with gcc); this module only marshals numpy arrays.
"""
from .oracle import (  # noqa: F401
    OracleParams,
    OracleSolver,
    OracleSim,
    build,
    lib,
    params_from_workload,
)
