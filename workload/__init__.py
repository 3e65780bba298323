"""Seeded synthetic inputs for the fermion-determinant path.

This module only *builds inputs*: the honeycomb hopping matrix, the auxiliary
field samples and the named workload configurations.  It holds none of the
method's arithmetic, so both the CPU oracle and the GPU path may use it.
"""
from .honeycomb import (  # noqa: F401
    honeycomb_hopping,
    honeycomb_site,
    sample_phi,
    uniform_phi,
    Workload,
    WORKLOADS,
    batched_mix,
    hmc_batch,
)
