"""ctypes binding of ``libnnqs_eloc.so`` (argument marshalling only).

Every entry point of ``include/nnqs_eloc.h`` is declared here with the same
name.  Device buffers are torch tensors on the current HIP device; streams
are torch streams.  Nothing here computes any part of the method.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libnnqs_eloc.so")

_c_void_p = ctypes.c_void_p
_i32, _i64, _u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
_f64 = ctypes.c_double

# (restype, argtypes) of every exported symbol.
SIGNATURES = {
    "nnqs_last_error": (ctypes.c_char_p, []),
    "nnqs_version": (ctypes.c_char_p, []),
    "nnqs_system_create": (_i32, [ctypes.POINTER(_c_void_p), _i32, _i32, _i32, _c_void_p, _c_void_p, _f64]),
    "nnqs_system_destroy": (_i32, [_c_void_p]),
    "nnqs_connection_count": (_i64, [_c_void_p]),
    "nnqs_table_create": (_i32, [ctypes.POINTER(_c_void_p), _c_void_p, _i64]),
    "nnqs_table_destroy": (_i32, [_c_void_p]),
    "nnqs_table_build": (_i32, [_c_void_p, _c_void_p, _c_void_p, _c_void_p, _i64, _u32, _c_void_p]),
    "nnqs_table_export": (_i32, [_c_void_p, _c_void_p, _c_void_p, _c_void_p, ctypes.POINTER(_i64), _c_void_p]),
    "nnqs_table_status": (_i32, [_c_void_p, _c_void_p]),
    "nnqs_connections": (_i32, [_c_void_p, _c_void_p, _i64, _c_void_p, _c_void_p, _c_void_p, _c_void_p, _u32,
                                _c_void_p]),
    "nnqs_eloc_table": (_i32, [_c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p, _i64, _c_void_p,
                               _c_void_p, _u32, _c_void_p]),
    "nnqs_energy": (_i32, [_c_void_p, _c_void_p, _c_void_p, _i64, _c_void_p, _c_void_p]),
    "nnqs_energy_noalloc": (_i32, [_c_void_p, _c_void_p, _i64, _c_void_p, _c_void_p]),
    "nnqs_screen_judge": (_i32, [_c_void_p, _c_void_p, _c_void_p, _c_void_p, _i64, _i32, _f64,
                                 ctypes.POINTER(_f64), ctypes.POINTER(_i32), _c_void_p]),
    "nnqs_timing_enable": (_i32, [_i32]),
    "nnqs_bas": (_i32, [_c_void_p, _i32, ctypes.c_uint64, ctypes.c_uint64, _i64, _c_void_p, _c_void_p, _c_void_p,
                        _c_void_p, ctypes.POINTER(_i64), _c_void_p]),
    "nnqs_tune_key": (_i32, [_c_void_p, _i64, ctypes.c_char_p, _i64]),
    "nnqs_tune_cache_lookup": (_i32, [ctypes.c_char_p, ctypes.c_char_p, _c_void_p, ctypes.POINTER(_f64),
                                      ctypes.POINTER(_i32)]),
    "nnqs_tune_cache_store": (_i32, [ctypes.c_char_p, ctypes.c_char_p, _c_void_p, _f64]),
    "nnqs_model_grad": (_i32, [_c_void_p, _c_void_p, _i64, _c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p,
                               _c_void_p]),
    "nnqs_vmc_gradient": (_i32, [_c_void_p, _c_void_p, _c_void_p, _c_void_p, _i64, _c_void_p, _c_void_p,
                                 _c_void_p]),
    "nnqs_lr_schedule": (_f64, [_i64, _i32, _i32]),
    "nnqs_model_adamw_step": (_i32, [_c_void_p, _c_void_p, _i64, _f64, _f64, _f64, _f64, _f64, _c_void_p,
                                     _c_void_p, _c_void_p]),
    "nnqs_model_get_weights": (_i32, [_c_void_p, _c_void_p, _c_void_p]),
    "nnqs_batch_model_create": (_i32, [ctypes.POINTER(_c_void_p), _c_void_p, _i32]),
    "nnqs_batch_model_destroy": (_i32, [_c_void_p]),
    "nnqs_batch_model_run": (_i32, [_c_void_p, _c_void_p]),
    "nnqs_batch_model_capture": (_i32, [_c_void_p, _c_void_p]),
    "nnqs_batch_model_launch": (_i32, [_c_void_p, _c_void_p]),
    "nnqs_timing_read": (_i32, [ctypes.c_char_p, ctypes.POINTER(_f64), ctypes.POINTER(_i64)]),
    "nnqs_table_set_tune": (_i32, [_c_void_p, _c_void_p]),
    "nnqs_table_get_tune": (_i32, [_c_void_p, _c_void_p]),
    "nnqs_model_weight_count": (_i64, [_c_void_p]),
    "nnqs_model_create": (_i32, [ctypes.POINTER(_c_void_p), _c_void_p, _c_void_p]),
    "nnqs_model_destroy": (_i32, [_c_void_p]),
    "nnqs_model_logpsi": (_i32, [_c_void_p, _c_void_p, _i64, _i32, _c_void_p, _c_void_p, _c_void_p]),
    "nnqs_eloc_model": (_i32, [_c_void_p, _c_void_p, _c_void_p, _c_void_p, _i32, _c_void_p, _c_void_p, _i64,
                               _c_void_p, _c_void_p, _c_void_p, _u32, _c_void_p]),
    "nnqs_screen_weight_count": (_i64, [_i32, _i32]),
    "nnqs_screen_create": (_i32, [ctypes.POINTER(_c_void_p), _i32, _i32, _c_void_p]),
    "nnqs_screen_destroy": (_i32, [_c_void_p]),
    "nnqs_screen_get_weights": (_i32, [_c_void_p, _c_void_p, _c_void_p]),
    "nnqs_screen_get_state": (_i32, [_c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p]),
    "nnqs_screen_set_state": (_i32, [_c_void_p, _c_void_p, _c_void_p, _i64, _c_void_p]),
    "nnqs_screen_forward": (_i32, [_c_void_p, _c_void_p, _c_void_p, _i64, _i32, _c_void_p, _c_void_p]),
    "nnqs_screen_gradient": (_i32, [_c_void_p, _c_void_p, _c_void_p, _c_void_p, _i64, _i32, _c_void_p, _c_void_p,
                                    _c_void_p]),
    "nnqs_screen_adam_step": (_i32, [_c_void_p, _c_void_p, _f64, _f64, _f64, _f64, _c_void_p]),
    "nnqs_table_autotune": (_i32, [_c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p, _i64, _c_void_p, _i32,
                                   _c_void_p, _c_void_p, _c_void_p]),
    "nnqs_pauli_build_host": (_i32, [_i32, _c_void_p, _c_void_p, _f64, _c_void_p, _c_void_p, _c_void_p, _c_void_p,
                                     _c_void_p, _c_void_p]),
    "nnqs_pauli_create": (_i32, [ctypes.POINTER(_c_void_p), _c_void_p]),
    "nnqs_pauli_destroy": (_i32, [_c_void_p]),
    "nnqs_pauli_info": (_i32, [_c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p]),
    "nnqs_eloc_pauli": (_i32, [_c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p, _c_void_p, _i64, _c_void_p,
                               _c_void_p, _u32, _c_void_p]),
    "nnqs_batch_create": (_i32, [ctypes.POINTER(_c_void_p), _c_void_p, _i32]),
    "nnqs_batch_destroy": (_i32, [_c_void_p]),
    "nnqs_batch_run": (_i32, [_c_void_p, _c_void_p]),
    "nnqs_batch_capture": (_i32, [_c_void_p, _c_void_p]),
    "nnqs_batch_launch": (_i32, [_c_void_p, _c_void_p]),
    "nnqs_batch_set_tune": (_i32, [_c_void_p, _c_void_p]),
    "nnqs_batch_get_tune": (_i32, [_c_void_p, _c_void_p]),
    "nnqs_batch_autotune": (_i32, [_c_void_p, _i32, _c_void_p, _c_void_p, _c_void_p]),
}

STATUS_NAMES = {0: "NNQS_OK", -1: "NNQS_EINVAL", -2: "NNQS_EDUP", -3: "NNQS_ECONSERVE", -4: "NNQS_ERANGE",
                -5: "NNQS_ENOMEM", -6: "NNQS_EHIP", -7: "NNQS_EUNSUPPORTED"}
NNQS_VALIDATE = 1


class NNQSError(RuntimeError):
    def __init__(self, code: int, message: str):
        self.code = code
        super().__init__(f"{STATUS_NAMES.get(code, code)}: {message}")


class Tune(ctypes.Structure):
    _fields_ = [("waves_per_block", _i32), ("blocks_per_cu", _i32), ("filter_log2_bits", _i32),
                ("splitter_levels", _i32), ("search", _i32), ("tile_samples", _i32)]


class BatchItem(ctypes.Structure):
    _fields_ = [("system", _c_void_p), ("table", _c_void_p), ("model", _c_void_p), ("keys", _c_void_p),
                ("counts", _c_void_p), ("logabs", _c_void_p), ("phase", _c_void_p), ("n", _i64),
                ("eloc", _c_void_p), ("energy", _c_void_p)]


class BatchModelItem(ctypes.Structure):
    _fields_ = [("system", _c_void_p), ("model", _c_void_p), ("keys", _c_void_p), ("counts", _c_void_p),
                ("n", _i64), ("eloc", _c_void_p), ("energy", _c_void_p)]


class ModelDesc(ctypes.Structure):
    _fields_ = [("n_orb", _i32), ("d_model", _i32), ("n_layers", _i32), ("n_heads", _i32), ("d_ff", _i32),
                ("phase_hidden", _i32), ("n_up", _i32), ("n_dn", _i32)]


class Stats(ctypes.Structure):
    _fields_ = [("connections", _i64), ("evaluated", _i64), ("refined", _i64), ("evaluated_class", _i64 * 4),
                ("evaluated_rows", _i64), ("evaluated_keys", _i64), ("evaluated_distinct", _i64)]


class ElocOpts(ctypes.Structure):
    _fields_ = [("skip_nats", _f64), ("skip_rule", _i32), ("refine_nats", _f64), ("screen_precision", _i32),
                ("dedup", _i32)]


NNQS_SKIP_RATIO = 0
NNQS_SKIP_CONTRIBUTION = 1


NNQS_FP64 = 0
NNQS_BF16 = 1
NNQS_FP32 = 2
NNQS_FP8 = 3

_lib = None


def load():
    """Load the built library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2306_16705_amd.build.build() "
                          "(hipcc --offload-arch=gfx950)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(code: int) -> None:
    if code != 0:
        msg = load().nnqs_last_error().decode(errors="replace")
        raise NNQSError(code, msg)
