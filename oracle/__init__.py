"""FP64 CPU oracle for the local energy (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this package.  It shares no code with the HIP library.
"""
from .oracle import (  # noqa: F401
    build,
    lib_path,
    n_connections,
    hxx,
    connections,
    sort_table,
    eloc_table,
    energy,
    net_order,
    pack_net,
    net_conditionals,
    net_logpsi,
    eloc_model,
    screen_size,
    screen_forward,
    screen_loss_grad,
    adam_step,
    philox4x32_10,
    bas_uniform,
    bas,
)
