"""Seeded synthetic inputs shared by the oracle and the HIP path.

This package only draws random numbers and places them into arrays: model
parameters of a Frenkel-Holstein exciton-vibration chain, the chain layout,
raw (non-canonical) initial MPS tensors, and random tensors for unit tests.
It performs none of the time-evolution arithmetic (no contraction, no QR, no
exponential); each side does that on its own.
"""

from .fmo import (  # noqa: F401
    ChainParams,
    draw_params,
    chain_sites,
    bond_dims,
    initial_mps_raw,
    workload,
    WORKLOADS,
)
from .randt import random_complex, random_mpo_like  # noqa: F401
