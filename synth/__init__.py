"""Seeded synthetic inputs shared by the FP64 oracle and the HIP path.

This package draws random numbers and packs bit strings; it holds none of the
local-energy arithmetic.  Both sides consume exactly the arrays produced here.
"""
from .gen import (  # noqa: F401
    SEED_ROOT,
    pack_occupations,
    unpack_keys,
    hf_key,
    all_determinants,
    integrals,
    geometric_samples,
    sample_amplitudes,
    sample_counts,
    config_inputs,
    batched_system_specs,
    transformer_weights,
    TransformerShape,
)
