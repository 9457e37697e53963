"""ctypes binding of the plain-C FP64 oracle (test infrastructure only).

The C source ``nnqs_oracle.c`` follows the paper's definitions: Eq. 4 (local
energy), Eq. 6 (sample mean over unique samples weighted by their counts,
Section 3.1), Eq. 9 (second-quantised Hamiltonian) and Section 3.4 items 4-5
(sample-aware evaluation over a sorted table of packed integer keys).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = [os.path.join(_HERE, "nnqs_oracle.c")]
_LIB = os.path.join(_HERE, "libnnqs_oracle.so")
_lib = None

_u64p = ctypes.POINTER(ctypes.c_uint64)
_f64p = ctypes.POINTER(ctypes.c_double)
_i8p = ctypes.POINTER(ctypes.c_int8)
_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_f32p = ctypes.POINTER(ctypes.c_float)


def lib_path() -> str:
    return _LIB


def build() -> str:
    """Compile the oracle with gcc (-O2, OpenMP, no fast-math)."""
    cmd = ["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-Wall", "-Wno-unknown-pragmas",
           "-o", _LIB + ".tmp", *_SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_LIB + ".tmp", _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or any(os.path.getmtime(s) > os.path.getmtime(_LIB) for s in _SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    lib.ora_n_connections.restype = ctypes.c_int64
    lib.ora_n_connections.argtypes = [ctypes.c_int] * 3
    lib.ora_hxx.restype = ctypes.c_double
    lib.ora_hxx.argtypes = [ctypes.c_int, _f64p, _f64p, ctypes.c_double, _u64p, _u64p,
                            ctypes.POINTER(ctypes.c_int)]
    lib.ora_connections.restype = ctypes.c_int64
    lib.ora_connections.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _f64p, _f64p, ctypes.c_double,
                                    _u64p, _u64p, _i8p, _u8p, _f64p]
    lib.ora_sort_table.restype = ctypes.c_int
    lib.ora_sort_table.argtypes = [_u64p, _f64p, _f64p, ctypes.c_int64, _u64p, _f64p, _f64p]
    lib.ora_eloc_table.restype = ctypes.c_int
    lib.ora_eloc_table.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, _f64p, _f64p, ctypes.c_double,
                                   _u64p, _f64p, _f64p, ctypes.c_int64,
                                   _u64p, _f64p, _f64p, ctypes.c_int64, _f64p, _f64p, ctypes.c_int]
    lib.ora_energy.restype = None
    lib.ora_energy.argtypes = [_u32p, _f64p, ctypes.c_int64, _f64p]
    _i = ctypes.c_int
    lib.ora_net_size.restype = ctypes.c_int64
    lib.ora_net_size.argtypes = [_i] * 6
    lib.ora_net_conditionals.restype = None
    lib.ora_net_conditionals.argtypes = [_i] * 8 + [_f64p, _u64p, _f64p]
    lib.ora_net_logpsi.restype = None
    lib.ora_net_logpsi.argtypes = [_i] * 8 + [_f64p, _u64p, ctypes.c_int64, _f64p, _f64p, _i]
    lib.ora_eloc_model.restype = ctypes.c_int
    lib.ora_eloc_model.argtypes = [_i, _i, _i, _f64p, _f64p, ctypes.c_double, _i, _i, _i, _i, _i, _f64p,
                                   _u64p, ctypes.c_int64, _f64p, _f64p, _i]
    lib.ora_screen_size.restype = ctypes.c_int64
    lib.ora_screen_size.argtypes = [_i, _i]
    lib.ora_screen_forward.restype = None
    lib.ora_screen_forward.argtypes = [_i, _i, _f64p, _u64p, _u8p, ctypes.c_int64, _f64p]
    lib.ora_screen_loss_grad.restype = ctypes.c_double
    lib.ora_screen_loss_grad.argtypes = [_i, _i, _f64p, _u64p, _u8p, _f64p, ctypes.c_int64, _f64p]
    lib.ora_adam_step.restype = None
    lib.ora_adam_step.argtypes = [_f64p, _f64p, _f64p, _f64p, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                  ctypes.c_double, ctypes.c_double, _i]
    lib.ora_philox4x32_10.restype = None
    lib.ora_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
    lib.ora_bas_uniform.restype = ctypes.c_double
    lib.ora_bas_uniform.argtypes = [ctypes.c_uint64, _i, ctypes.c_uint64]
    lib.ora_bas.restype = ctypes.c_int64
    lib.ora_bas.argtypes = [_i] * 8 + [_f64p, ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64, _u64p, _u32p, _f64p]
    _lib = lib
    return lib


def _p(a: np.ndarray, t):
    return a.ctypes.data_as(t)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def n_connections(K: int, n_up: int, n_dn: int) -> int:
    return int(_load().ora_n_connections(K, n_up, n_dn))


def hxx(K, h, g, e_core, x, xp):
    """``<x'|H|x>`` and the sign of the excitation operator on ``x``."""
    h, g = _c(h, np.float64), _c(g, np.float64)
    x, xp = _c(x, np.uint64), _c(xp, np.uint64)
    s = ctypes.c_int(0)
    v = _load().ora_hxx(K, _p(h, _f64p), _p(g, _f64p), float(e_core), _p(x, _u64p), _p(xp, _u64p),
                        ctypes.byref(s))
    return v, s.value


def connections(K, n_up, n_dn, h, g, e_core, x):
    """Canonical-order connections of one configuration: ``(xp[C,2], sign[C],
    exc[C,4], hxx[C])``."""
    lib = _load()
    C = n_connections(K, n_up, n_dn)
    h, g, x = _c(h, np.float64), _c(g, np.float64), _c(x, np.uint64)
    xp = np.zeros((C, 2), np.uint64)
    sign = np.zeros(C, np.int8)
    exc = np.zeros((C, 4), np.uint8)
    hv = np.zeros(C, np.float64)
    r = lib.ora_connections(K, n_up, n_dn, _p(h, _f64p), _p(g, _f64p), float(e_core), _p(x, _u64p),
                            _p(xp, _u64p), _p(sign, _i8p), _p(exc, _u8p), _p(hv, _f64p))
    if r < 0:
        raise ValueError("configuration violates the particle numbers")
    assert r == C
    return xp, sign, exc, hv


def sort_table(keys, logabs, phase):
    """Sorted copy of a table (qsort, unsigned 128-bit order, word 1 major)
    and whether its keys are unique."""
    keys, logabs, phase = _c(keys, np.uint64), _c(logabs, np.float64), _c(phase, np.float64)
    n = logabs.shape[0]
    ko = np.zeros((n, 2), np.uint64)
    lo = np.zeros(n, np.float64)
    po = np.zeros(n, np.float64)
    u = _load().ora_sort_table(_p(keys, _u64p), _p(logabs, _f64p), _p(phase, _f64p), n,
                               _p(ko, _u64p), _p(lo, _f64p), _p(po, _f64p))
    return ko, lo, po, bool(u)


def eloc_table(K, n_up, n_dn, h, g, e_core, tkeys, tlogabs, tphase, keys, logabs, phase,
               nthreads: int = 0, with_absum: bool = False):
    """Sample-aware local energies ``complex128[n]`` (and optionally the
    per-sample scale ``sum |H| |psi'/psi|``)."""
    lib = _load()
    h, g = _c(h, np.float64), _c(g, np.float64)
    tkeys, tlogabs, tphase = _c(tkeys, np.uint64), _c(tlogabs, np.float64), _c(tphase, np.float64)
    keys, logabs, phase = _c(keys, np.uint64), _c(logabs, np.float64), _c(phase, np.float64)
    n = logabs.shape[0]
    out = np.zeros((n, 2), np.float64)
    ab = np.zeros(n, np.float64)
    r = lib.ora_eloc_table(K, n_up, n_dn, _p(h, _f64p), _p(g, _f64p), float(e_core),
                           _p(tkeys, _u64p), _p(tlogabs, _f64p), _p(tphase, _f64p), tlogabs.shape[0],
                           _p(keys, _u64p), _p(logabs, _f64p), _p(phase, _f64p), n,
                           _p(out, _f64p), _p(ab, _f64p), int(nthreads))
    if r < 0:
        raise ValueError("a sample violates the particle numbers")
    e = out[:, 0] + 1j * out[:, 1]
    return (e, ab) if with_absum else e


def energy(counts, eloc):
    """``[E_re, E_im, sum_w, var]`` of Eq. 6 with occurrence counts."""
    counts = _c(counts, np.uint32)
    e = np.ascontiguousarray(np.stack([np.real(eloc), np.imag(eloc)], axis=1), dtype=np.float64)
    out = np.zeros(4, np.float64)
    _load().ora_energy(_p(counts, _u32p), _p(e, _f64p), counts.shape[0], _p(out, _f64p))
    return out


# ------------------------------------------------------------------ networks
def net_order(L: int):
    """Names of the network weights in the order the C oracle reads them."""
    names = ["tok_emb", "pos_emb"]
    for l in range(L):
        names += [f"l{l}.{k}" for k in ("ln1_g", "ln1_b", "wq", "bq", "wk", "bk", "wv", "bv", "wo", "bo",
                                        "ln2_g", "ln2_b", "w1", "b1", "w2", "b2")]
    names += ["lnf_g", "lnf_b", "head_w", "head_b", "logit_bias", "ph_w1", "ph_b1", "ph_w2", "ph_b2",
              "ph_w3", "ph_b3"]
    return names


def pack_net(weights: dict, shape) -> np.ndarray:
    """Flatten the weight dict into the oracle's float64 layout."""
    flat = np.concatenate([np.asarray(weights[k], dtype=np.float64).ravel() for k in net_order(shape.n_layers)])
    n = _load().ora_net_size(shape.K, shape.d_model, shape.n_layers, shape.n_heads, shape.d_ff, shape.phase_hidden)
    assert flat.size == n, (flat.size, n)
    return np.ascontiguousarray(flat)


def _dims(shape):
    return (shape.K, shape.d_model, shape.n_layers, shape.n_heads, shape.d_ff, shape.phase_hidden)


def net_conditionals(weights, shape, n_up, n_dn, x):
    """Masked conditional log-probabilities ``[K, 4]`` of one configuration."""
    w = pack_net(weights, shape)
    x = _c(x, np.uint64)
    out = np.zeros((shape.K, 4), np.float64)
    _load().ora_net_conditionals(*_dims(shape), n_up, n_dn, _p(w, _f64p), _p(x, _u64p), _p(out, _f64p))
    return out


def net_logpsi(weights, shape, n_up, n_dn, keys, nthreads: int = 0):
    """``(log|psi|, phase)`` of every configuration in ``keys [n, 2]``."""
    w = pack_net(weights, shape)
    keys = _c(keys, np.uint64).reshape(-1, 2)
    n = keys.shape[0]
    la = np.zeros(n, np.float64)
    ph = np.zeros(n, np.float64)
    _load().ora_net_logpsi(*_dims(shape), n_up, n_dn, _p(w, _f64p), _p(keys, _u64p), n, _p(la, _f64p),
                           _p(ph, _f64p), int(nthreads))
    return la, ph


def eloc_model(K, n_up, n_dn, h, g, e_core, weights, shape, keys, nthreads: int = 0, with_absum: bool = False):
    """Full local energies with every x' amplitude from the networks."""
    w = pack_net(weights, shape)
    h, g = _c(h, np.float64), _c(g, np.float64)
    keys = _c(keys, np.uint64).reshape(-1, 2)
    n = keys.shape[0]
    out = np.zeros((n, 2), np.float64)
    ab = np.zeros(n, np.float64)
    d = _dims(shape)
    r = _load().ora_eloc_model(K, n_up, n_dn, _p(h, _f64p), _p(g, _f64p), float(e_core), d[1], d[2], d[3], d[4],
                               d[5], _p(w, _f64p), _p(keys, _u64p), n, _p(out, _f64p), _p(ab, _f64p), int(nthreads))
    if r < 0:
        raise ValueError("a sample violates the particle numbers")
    e = out[:, 0] + 1j * out[:, 1]
    return (e, ab) if with_absum else e


# ------------------------------------------------------------------- screen
def screen_size(N: int, H: int) -> int:
    return int(_load().ora_screen_size(N, H))


def screen_forward(N, H, w, keys, exc):
    w = _c(w, np.float64)
    keys = _c(keys, np.uint64).reshape(-1, 2)
    exc = _c(exc, np.uint8).reshape(-1, 4)
    out = np.zeros(keys.shape[0], np.float64)
    _load().ora_screen_forward(N, H, _p(w, _f64p), _p(keys, _u64p), _p(exc, _u8p), keys.shape[0], _p(out, _f64p))
    return out


def screen_loss_grad(N, H, w, keys, exc, target):
    w = _c(w, np.float64)
    keys = _c(keys, np.uint64).reshape(-1, 2)
    exc = _c(exc, np.uint8).reshape(-1, 4)
    target = _c(target, np.float64)
    g = np.zeros(screen_size(N, H), np.float64)
    loss = _load().ora_screen_loss_grad(N, H, _p(w, _f64p), _p(keys, _u64p), _p(exc, _u8p), _p(target, _f64p),
                                        keys.shape[0], _p(g, _f64p))
    return float(loss), g


def adam_step(w, grad, m, v, lr, beta1, beta2, eps, t):
    """In-place Adam update of float64 arrays w, m, v."""
    for a in (w, grad, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    _load().ora_adam_step(_p(w, _f64p), _p(grad, _f64p), _p(m, _f64p), _p(v, _f64p), w.size, lr, beta1, beta2,
                          eps, int(t))


# ------------------------------------------- batch autoregressive sampling
def philox4x32_10(ctr, key):
    """Philox4x32-10 of a 4-word counter and a 2-word key (four uint32 words)."""
    c = _c(ctr, np.uint32)
    k = _c(key, np.uint32)
    out = np.zeros(4, np.uint32)
    _load().ora_philox4x32_10(_p(c, _u32p), _p(k, _u32p), _p(out, _u32p))
    return out


def bas_uniform(seed: int, s: int, i: int) -> float:
    return float(_load().ora_bas_uniform(int(seed), int(s), int(i)))


def bas(weights, shape, n_up, n_dn, n_samples: int, seed: int, capacity: int = 1 << 20):
    """Batch autoregressive sampling (Section 3.1) with the FP64 network:
    ``(keys [m, 2], counts [m] uint32, logabs [m])`` of the unique samples in
    generation order."""
    w = pack_net(weights, shape)
    keys = np.zeros((capacity, 2), np.uint64)
    counts = np.zeros(capacity, np.uint32)
    la = np.zeros(capacity, np.float64)
    m = _load().ora_bas(*_dims(shape), n_up, n_dn, _p(w, _f64p), int(n_samples), int(seed), int(capacity),
                        _p(keys, _u64p), _p(counts, _u32p), _p(la, _f64p))
    if m < 0:
        raise ValueError("capacity exceeded")
    return keys[:m].copy(), counts[:m].copy(), la[:m].copy()
