"""MI355X-native local-energy library for neural-network quantum states.

Python face of ``libnnqs_eloc.so``: thin wrappers with the names of the C ABI
(``include/nnqs_eloc.h``) that marshal torch device tensors and streams.
All computation happens in the HIP kernels of the library; there is no
fallback path.
"""
from .api import (  # noqa: F401
    Batch,
    BatchModel,
    NNQSError,
    NNQS_BF16,
    NNQS_FP32,
    NNQS_FP8,
    NNQS_FP64,
    NNQS_SKIP_CONTRIBUTION,
    NNQS_SKIP_RATIO,
    NNQS_VALIDATE,
    Model,
    Pauli,
    Screen,
    System,
    Table,
    bas,
    connections,
    eloc_model,
    eloc_pauli,
    eloc_table,
    energy,
    energy_noalloc,
    lr_schedule,
    model_adamw_step,
    model_get_weights,
    model_grad,
    model_logpsi,
    pauli_build_host,
    timing_enable,
    timing_read,
    tune_cache_lookup,
    tune_cache_store,
    tune_key,
    version,
    vmc_gradient,
)
