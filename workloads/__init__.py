"""Seeded synthetic inputs shared by the HIP path's tests/bench and the CPU oracle.

This package draws random numbers and lays them out as little-endian 32-bit
limb arrays; it holds none of the commit/accumulate arithmetic (no field
multiplication, no curve operation, no transform).  Both sides of every parity
check receive the same bytes from here.
"""
from .generators import (  # noqa: F401
    FR_MODULUS,
    TAU_SEED,
    CONFIG_SEEDS,
    rng_for,
    uniform_fr,
    quantized_fr,
    quantized_values,
    log_uniform_sizes,
    poisson_arrivals,
    tau_scalar,
    ints_to_limbs,
    limbs_to_ints,
    commit_job_eval_sizes,
)
