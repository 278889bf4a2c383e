"""Seeded synthetic inputs shared by the oracle-side tests and the HIP path.

This package holds workload descriptions (lattice sizes, droplet geometry, material
parameters derived from the paper's dimensionless groups) and seeded random fields.
It holds none of the coupled step's arithmetic and imports neither the oracle nor
the HIP binding.
"""
from .workloads import (  # noqa: F401
    Workload,
    channel_drive,
    h0_from_bond,
    sigma_from_capillary,
    single_channel_small,
    single_channel_large,
    open_channel_small,
    open_channel_paper,
    adjoint_channel,
    regime_sweep_batch,
    adjoint_batch,
    random_phase_fields,
)
