"""Object wrappers over the C ABI (argument marshalling only)."""
from __future__ import annotations

import ctypes
import hashlib
import os

import numpy as np
import torch

from . import _lib as L
from ._lib import (NNQS_BF16, NNQS_FP8, NNQS_FP32, NNQS_FP64, NNQS_SKIP_CONTRIBUTION, NNQS_SKIP_RATIO,  # noqa: F401
                   NNQS_VALIDATE, ModelDesc, NNQSError, Stats, Tune)

_KEY_DTYPES = (torch.int64, torch.uint64)


def version() -> str:
    return L.load().nnqs_version().decode()


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _need(t, name, dtypes, shape=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype not in dtypes:
        raise TypeError(f"{name} has dtype {t.dtype}, expected one of {dtypes}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    return t


class System:
    """Hamiltonian of Eq. 9 on the current device (``nnqs_system_*``)."""

    def __init__(self, n_spin_orb: int, n_up: int, n_dn: int, h, g, e_core: float = 0.0):
        K = n_spin_orb // 2
        h = np.ascontiguousarray(h, dtype=np.float64)
        g = np.ascontiguousarray(g, dtype=np.float64)
        if h.shape != (K, K) or g.shape != (K, K, K, K):
            raise ValueError("h must be [K, K] and g [K, K, K, K]")
        self._lib = L.load()
        out = ctypes.c_void_p()
        L.check(self._lib.nnqs_system_create(ctypes.byref(out), n_spin_orb, n_up, n_dn,
                                             h.ctypes.data_as(ctypes.c_void_p), g.ctypes.data_as(ctypes.c_void_p),
                                             float(e_core)))
        self.handle = out
        self.n_spin_orb, self.n_up, self.n_dn, self.K = n_spin_orb, n_up, n_dn, K

    @property
    def connection_count(self) -> int:
        return int(self._lib.nnqs_connection_count(self.handle))

    def close(self):
        if getattr(self, "handle", None):
            self._lib.nnqs_system_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Table:
    """Sorted unique-sample table (``nnqs_table_*``)."""

    def __init__(self, system: System, capacity: int):
        self._lib = L.load()
        self.system = system
        out = ctypes.c_void_p()
        L.check(self._lib.nnqs_table_create(ctypes.byref(out), system.handle, int(capacity)))
        self.handle = out
        self.capacity = int(capacity)

    def build(self, keys, logabs, phase, validate: bool = False, stream=None):
        n = keys.shape[0]
        _need(keys, "keys", _KEY_DTYPES, (n, 2))
        _need(logabs, "logabs", (torch.float64,), (n,))
        _need(phase, "phase", (torch.float64,), (n,))
        L.check(self._lib.nnqs_table_build(self.handle, _ptr(keys), _ptr(logabs), _ptr(phase), n,
                                           NNQS_VALIDATE if validate else 0, _stream(stream)))
        return self

    def export(self, stream=None):
        dev = torch.device("cuda", torch.cuda.current_device())
        keys = torch.empty((self.capacity, 2), dtype=torch.int64, device=dev)
        la = torch.empty(self.capacity, dtype=torch.float64, device=dev)
        ph = torch.empty(self.capacity, dtype=torch.float64, device=dev)
        n = ctypes.c_int64(0)
        L.check(self._lib.nnqs_table_export(self.handle, _ptr(keys), _ptr(la), _ptr(ph), ctypes.byref(n),
                                            _stream(stream)))
        m = n.value
        return keys[:m], la[:m], ph[:m]

    def status(self, stream=None) -> int:
        return int(self._lib.nnqs_table_status(self.handle, _stream(stream)))

    def set_tune(self, waves_per_block=0, blocks_per_cu=0, filter_log2_bits=0, splitter_levels=0, search=0,
                 tile_samples=0):
        t = Tune(waves_per_block, blocks_per_cu, filter_log2_bits, splitter_levels, search, tile_samples)
        L.check(self._lib.nnqs_table_set_tune(self.handle, ctypes.byref(t)))

    def get_tune(self) -> dict:
        t = Tune()
        L.check(self._lib.nnqs_table_get_tune(self.handle, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in Tune._fields_}

    def autotune(self, keys, logabs, phase, reps: int = 2, eloc=None, cache_path: str | None = None, stream=None):
        """Times the candidate schedules of ``nnqs_eloc_table`` on these
        samples, keeps the fastest (the table is left built from them) and
        returns ``(tune dict, best ms)``.  With ``cache_path`` (default: the
        ``NNQS_TUNE_CACHE`` environment variable) a schedule stored there for
        this workload's key is used without timing, and a newly timed one is
        stored (``nnqs_tune_cache_*``)."""
        n = keys.shape[0]
        _need(keys, "keys", _KEY_DTYPES, (n, 2))
        _need(logabs, "logabs", (torch.float64,), (n,))
        _need(phase, "phase", (torch.float64,), (n,))
        t = Tune()
        ms = ctypes.c_double()
        key = None
        if cache_path is None:
            cache_path = os.environ.get("NNQS_TUNE_CACHE") or None
        if cache_path is not None:
            key = tune_key(self.system, n)
            found = ctypes.c_int32(0)
            L.check(self._lib.nnqs_tune_cache_lookup(cache_path.encode(), key.encode(), ctypes.byref(t),
                                                     ctypes.byref(ms), ctypes.byref(found)))
            if found.value:
                L.check(self._lib.nnqs_table_set_tune(self.handle, ctypes.byref(t)))
                self.build(keys, logabs, phase, stream=stream)
                return {f: getattr(t, f) for f, _ in Tune._fields_}, ms.value
        if eloc is None:
            eloc = torch.empty((n, 2), dtype=torch.float64, device=keys.device)
        L.check(self._lib.nnqs_table_autotune(self.system.handle, self.handle, _ptr(keys), _ptr(logabs), _ptr(phase),
                                              n, _ptr(eloc), int(reps), ctypes.byref(t), ctypes.byref(ms),
                                              _stream(stream)))
        if key is not None:
            L.check(self._lib.nnqs_tune_cache_store(cache_path.encode(), key.encode(), ctypes.byref(t), ms.value))
        return {f: getattr(t, f) for f, _ in Tune._fields_}, ms.value

    def close(self):
        if getattr(self, "handle", None):
            self._lib.nnqs_table_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def connections(system: System, keys, validate: bool = False, stream=None):
    """Canonical-order connections of every sample: dict of device tensors
    ``xprime [n, C, 2] int64``, ``sign [n, C] int8``, ``exc [n, C, 4] uint8``,
    ``hxx [n, C] float64`` (``nnqs_connections``)."""
    n = keys.shape[0]
    _need(keys, "keys", _KEY_DTYPES, (n, 2))
    C = system.connection_count
    dev = keys.device
    out = dict(xprime=torch.empty((n, C, 2), dtype=torch.int64, device=dev),
               sign=torch.empty((n, C), dtype=torch.int8, device=dev),
               exc=torch.empty((n, C, 4), dtype=torch.uint8, device=dev),
               hxx=torch.empty((n, C), dtype=torch.float64, device=dev))
    L.check(L.load().nnqs_connections(system.handle, _ptr(keys), n, _ptr(out["xprime"]), _ptr(out["sign"]),
                                      _ptr(out["exc"]), _ptr(out["hxx"]), NNQS_VALIDATE if validate else 0,
                                      _stream(stream)))
    return out


def eloc_table(system: System, table: Table, keys, counts, logabs, phase, eloc=None, energy=None,
               with_energy: bool = True, validate: bool = False, stream=None):
    """Sample-aware local energies (``nnqs_eloc_table``).  Returns
    ``(eloc [n, 2] float64, energy [4] float64 or None)``."""
    n = keys.shape[0]
    _need(keys, "keys", _KEY_DTYPES, (n, 2))
    _need(logabs, "logabs", (torch.float64,), (n,))
    _need(phase, "phase", (torch.float64,), (n,))
    if counts is not None:
        _need(counts, "counts", (torch.int32, torch.uint32), (n,))
    if eloc is None:
        eloc = torch.empty((n, 2), dtype=torch.float64, device=keys.device)
    _need(eloc, "eloc", (torch.float64,), (n, 2))
    if with_energy and energy is None:
        energy = torch.empty(4, dtype=torch.float64, device=keys.device)
    if energy is not None:
        _need(energy, "energy", (torch.float64,), (4,))
    L.check(L.load().nnqs_eloc_table(system.handle, table.handle, _ptr(keys), _ptr(counts), _ptr(logabs),
                                     _ptr(phase), n, _ptr(eloc), _ptr(energy) if with_energy else None,
                                     NNQS_VALIDATE if validate else 0, _stream(stream)))
    return eloc, (energy if with_energy else None)


def energy(table: Table, counts, eloc, out=None, stream=None):
    """Weighted energy of Eq. 6 from precomputed local energies (``nnqs_energy``)."""
    n = eloc.shape[0]
    _need(counts, "counts", (torch.int32, torch.uint32), (n,))
    _need(eloc, "eloc", (torch.float64,), (n, 2))
    if out is None:
        out = torch.empty(4, dtype=torch.float64, device=eloc.device)
    L.check(L.load().nnqs_energy(table.handle, _ptr(counts), _ptr(eloc), n, _ptr(out), _stream(stream)))
    return out


def energy_noalloc(counts, eloc, out=None, stream=None):
    """Weighted energy of Eq. 6 without a table, with the library's static
    per-GPU scratch (``nnqs_energy_noalloc``; allocates nothing)."""
    n = eloc.shape[0]
    _need(counts, "counts", (torch.int32, torch.uint32), (n,))
    _need(eloc, "eloc", (torch.float64,), (n, 2))
    if out is None:
        out = torch.empty(4, dtype=torch.float64, device=eloc.device)
    _need(out, "energy", (torch.float64,), (4,))
    L.check(L.load().nnqs_energy_noalloc(_ptr(counts), _ptr(eloc), n, _ptr(out), _stream(stream)))
    return out


# ------------------------------------------------------------------- model
_LAYER_KEYS = ("ln1_g", "ln1_b", "wq", "bq", "wk", "bk", "wv", "bv", "wo", "bo", "ln2_g", "ln2_b", "w1", "b1",
               "w2", "b2")


def pack_model_weights(weights: dict, n_layers: int) -> np.ndarray:
    """FP32 weights in the order ``nnqs_model_create`` documents."""
    order = ["tok_emb", "pos_emb"] + [f"l{l}.{k}" for l in range(n_layers) for k in _LAYER_KEYS]
    order += ["lnf_g", "lnf_b", "head_w", "head_b", "logit_bias", "ph_w1", "ph_b1", "ph_w2", "ph_b2", "ph_w3",
              "ph_b3"]
    return np.ascontiguousarray(np.concatenate([np.asarray(weights[k], np.float32).ravel() for k in order]))


class Model:
    """Amplitude transformer + phase MLP on the device (``nnqs_model_*``)."""

    def __init__(self, shape, n_up: int, n_dn: int, weights: dict):
        self._lib = L.load()
        self.desc = ModelDesc(shape.K, shape.d_model, shape.n_layers, shape.n_heads, shape.d_ff,
                              shape.phase_hidden, n_up, n_dn)
        flat = pack_model_weights(weights, shape.n_layers)
        count = self._lib.nnqs_model_weight_count(ctypes.byref(self.desc))
        if count != flat.size:
            raise ValueError(f"weight count {flat.size} does not match the model description ({count})")
        out = ctypes.c_void_p()
        L.check(self._lib.nnqs_model_create(ctypes.byref(out), ctypes.byref(self.desc),
                                            flat.ctypes.data_as(ctypes.c_void_p)))
        self.handle = out

    def close(self):
        if getattr(self, "handle", None):
            self._lib.nnqs_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def bas(model: Model, n_samples: int, seed: int, precision: int = NNQS_BF16, capacity: int = 1 << 20,
        with_phase: bool = True, stream=None):
    """Batch autoregressive sampling (``nnqs_bas``): ``(keys [m, 2] int64,
    counts [m] int32 (uint32 values), logabs [m], phase [m] or None)`` of the
    unique samples on the current device."""
    dev = torch.device("cuda", torch.cuda.current_device())
    keys = torch.empty((capacity, 2), dtype=torch.int64, device=dev)
    counts = torch.empty(capacity, dtype=torch.int32, device=dev)
    la = torch.empty(capacity, dtype=torch.float64, device=dev)
    ph = torch.empty(capacity, dtype=torch.float64, device=dev) if with_phase else None
    m = ctypes.c_int64()
    L.check(L.load().nnqs_bas(model.handle, int(precision), int(seed), int(n_samples), int(capacity), _ptr(keys),
                              _ptr(counts), _ptr(la), _ptr(ph), ctypes.byref(m), _stream(stream)))
    k = m.value
    return keys[:k], counts[:k], la[:k], (ph[:k] if ph is not None else None)


def tune_key(system: System, n: int) -> str:
    """Autotuner cache key of a sample-aware workload (``nnqs_tune_key``)."""
    buf = ctypes.create_string_buffer(256)
    L.check(L.load().nnqs_tune_key(system.handle, int(n), buf, 256))
    return buf.value.decode()


def tune_cache_lookup(path: str, key: str):
    """``(tune dict, ms)`` stored for ``key`` in the cache file, or None."""
    t = Tune()
    ms = ctypes.c_double()
    found = ctypes.c_int32(0)
    L.check(L.load().nnqs_tune_cache_lookup(path.encode(), key.encode(), ctypes.byref(t), ctypes.byref(ms),
                                            ctypes.byref(found)))
    return ({f: getattr(t, f) for f, _ in Tune._fields_}, ms.value) if found.value else None


def tune_cache_store(path: str, key: str, tune: dict, ms: float) -> None:
    """Stores a schedule for ``key`` in the cache file (``nnqs_tune_cache_store``)."""
    t = Tune(*(int(tune[f]) for f, _ in Tune._fields_))
    L.check(L.load().nnqs_tune_cache_store(path.encode(), key.encode(), ctypes.byref(t), float(ms)))


def model_grad(model: Model, keys, c_logabs, c_phase, grad=None, with_values: bool = False, stream=None):
    """FP64 weighted parameter gradient (``nnqs_model_grad``): device tensor
    ``grad [weight_count]`` (and ``(logabs, phase)`` of the same pass with
    ``with_values``)."""
    n = keys.shape[0]
    _need(keys, "keys", _KEY_DTYPES, (n, 2))
    _need(c_logabs, "c_logabs", (torch.float64,), (n,))
    _need(c_phase, "c_phase", (torch.float64,), (n,))
    nw = L.load().nnqs_model_weight_count(ctypes.byref(model.desc))
    if grad is None:
        grad = torch.empty(nw, dtype=torch.float64, device=keys.device)
    la = torch.empty(n, dtype=torch.float64, device=keys.device) if with_values else None
    ph = torch.empty(n, dtype=torch.float64, device=keys.device) if with_values else None
    L.check(L.load().nnqs_model_grad(model.handle, _ptr(keys), n, _ptr(c_logabs), _ptr(c_phase), _ptr(grad),
                                     _ptr(la), _ptr(ph), _stream(stream)))
    return (grad, la, ph) if with_values else grad


def vmc_gradient(model: Model, keys, counts, eloc, grad=None, energy=None, stream=None):
    """Eq. 7 gradient (``nnqs_vmc_gradient``): ``(grad [weight_count],
    energy [4])`` device tensors."""
    n = keys.shape[0]
    _need(keys, "keys", _KEY_DTYPES, (n, 2))
    _need(counts, "counts", (torch.int32,), (n,))
    _need(eloc, "eloc", (torch.float64,), (n, 2))
    nw = L.load().nnqs_model_weight_count(ctypes.byref(model.desc))
    if grad is None:
        grad = torch.empty(nw, dtype=torch.float64, device=keys.device)
    if energy is None:
        energy = torch.empty(4, dtype=torch.float64, device=keys.device)
    L.check(L.load().nnqs_vmc_gradient(model.handle, _ptr(keys), _ptr(counts), _ptr(eloc), n, _ptr(grad),
                                       _ptr(energy), _stream(stream)))
    return grad, energy


def lr_schedule(step: int, d_model: int, warmup: int = 4000) -> float:
    """Eq. 13 learning rate (``nnqs_lr_schedule``)."""
    return float(L.load().nnqs_lr_schedule(int(step), int(d_model), int(warmup)))


def model_adamw_step(model: Model, grad, step: int, lr: float, mom1, mom2, beta1: float = 0.9,
                     beta2: float = 0.999, eps: float = 1e-8, weight_decay: float = 0.01, stream=None):
    """One AdamW step of the model's FP64 weights (``nnqs_model_adamw_step``)."""
    nw = L.load().nnqs_model_weight_count(ctypes.byref(model.desc))
    for t, name in ((grad, "grad"), (mom1, "mom1"), (mom2, "mom2")):
        _need(t, name, (torch.float64,), (nw,))
    L.check(L.load().nnqs_model_adamw_step(model.handle, _ptr(grad), int(step), float(lr), float(beta1),
                                           float(beta2), float(eps), float(weight_decay), _ptr(mom1), _ptr(mom2),
                                           _stream(stream)))


def model_get_weights(model: Model, out=None, stream=None):
    """The model's FP64 weights as a device tensor (``nnqs_model_get_weights``)."""
    nw = L.load().nnqs_model_weight_count(ctypes.byref(model.desc))
    dev = torch.device("cuda", torch.cuda.current_device())
    if out is None:
        out = torch.empty(nw, dtype=torch.float64, device=dev)
    L.check(L.load().nnqs_model_get_weights(model.handle, _ptr(out), _stream(stream)))
    return out


def model_logpsi(model: Model, keys, precision: int = NNQS_FP64, logabs=None, phase=None, stream=None):
    """``(log|psi|, phase)`` device tensors for ``keys [n, 2]`` (``nnqs_model_logpsi``)."""
    n = keys.shape[0]
    _need(keys, "keys", _KEY_DTYPES, (n, 2))
    if logabs is None:
        logabs = torch.empty(n, dtype=torch.float64, device=keys.device)
    if phase is None:
        phase = torch.empty(n, dtype=torch.float64, device=keys.device)
    L.check(L.load().nnqs_model_logpsi(model.handle, _ptr(keys), n, int(precision), _ptr(logabs), _ptr(phase),
                                       _stream(stream)))
    return logabs, phase


def eloc_model(system: System, model: Model, keys, counts=None, precision: int = NNQS_FP64, eloc=None,
               energy=None, with_energy: bool = True, with_stats: bool = False, validate: bool = False,
               screen=None, skip_nats: float = 12.0, skip_rule: int = L.NNQS_SKIP_RATIO, refine_nats: float = 0.0,
               screen_precision: int = NNQS_BF16, dedup: bool = False, stream=None):
    """Full local energies with every x' from the network (``nnqs_eloc_model``).

    With a learned ``screen`` only connections kept by ``skip_rule`` at
    ``skip_nats`` go to the network; ``refine_nats > 0`` re-evaluates in FP64
    every connection whose first-pass contribution is at least
    ``exp(-refine_nats)`` Ha; ``dedup`` evaluates every distinct x' of a
    chunk once (BF16 / FP8).  Returns ``(eloc [n, 2], energy [4] or None,
    stats dict or None)``."""
    n = keys.shape[0]
    _need(keys, "keys", _KEY_DTYPES, (n, 2))
    if with_energy:
        _need(counts, "counts", (torch.int32, torch.uint32), (n,))
        if energy is None:
            energy = torch.empty(4, dtype=torch.float64, device=keys.device)
    if eloc is None:
        eloc = torch.empty((n, 2), dtype=torch.float64, device=keys.device)
    st = Stats()
    opts = L.ElocOpts(float(skip_nats), int(skip_rule), float(refine_nats), int(screen_precision), int(bool(dedup)))
    L.check(L.load().nnqs_eloc_model(system.handle, model.handle, screen.handle if screen is not None else None,
                                     ctypes.byref(opts), int(precision), _ptr(keys), _ptr(counts), n,
                                     _ptr(eloc), _ptr(energy) if with_energy else None,
                                     ctypes.byref(st) if with_stats else None, NNQS_VALIDATE if validate else 0,
                                     _stream(stream)))
    stats = ({"connections": st.connections, "evaluated": st.evaluated, "refined": st.refined,
              "evaluated_class": list(st.evaluated_class), "evaluated_rows": st.evaluated_rows,
              "evaluated_keys": st.evaluated_keys, "evaluated_distinct": st.evaluated_distinct}
             if with_stats else None)
    return eloc, (energy if with_energy else None), stats


# ------------------------------------------------------------- measurement
def timing_enable(enable: bool = True) -> None:
    """Start (and clear) or stop the library's event timing of its hot launches."""
    L.check(L.load().nnqs_timing_enable(1 if enable else 0))


def timing_read(kernel: str):
    """``(total ms, launches)`` of ``kernel`` since the last ``timing_enable``."""
    ms, cnt = ctypes.c_double(), ctypes.c_int64()
    L.check(L.load().nnqs_timing_read(kernel.encode(), ctypes.byref(ms), ctypes.byref(cnt)))
    return ms.value, cnt.value


# ------------------------------------------------------------------ screen
class Screen:
    """Learned screen MLP (``nnqs_screen_*``): FP64 master weights on the device."""

    def __init__(self, n_spin_orb: int, hidden: int, weights):
        self._lib = L.load()
        w = np.ascontiguousarray(weights, dtype=np.float64)
        cnt = self._lib.nnqs_screen_weight_count(n_spin_orb, hidden)
        if cnt != w.size:
            raise ValueError(f"screen needs {cnt} weights, got {w.size}")
        out = ctypes.c_void_p()
        L.check(self._lib.nnqs_screen_create(ctypes.byref(out), n_spin_orb, hidden, w.ctypes.data_as(ctypes.c_void_p)))
        self.handle = out
        self.n_spin_orb, self.hidden, self.count = n_spin_orb, hidden, int(cnt)

    def weights(self, stream=None) -> np.ndarray:
        out = np.empty(self.count, np.float64)
        L.check(self._lib.nnqs_screen_get_weights(self.handle, out.ctypes.data_as(ctypes.c_void_p), _stream(stream)))
        return out

    def state(self, stream=None):
        """Adam state ``(m, v, t)``: host copies of both moments and the step count."""
        m, v = np.empty(self.count, np.float64), np.empty(self.count, np.float64)
        t = ctypes.c_int64()
        L.check(self._lib.nnqs_screen_get_state(self.handle, m.ctypes.data_as(ctypes.c_void_p),
                                                v.ctypes.data_as(ctypes.c_void_p), ctypes.byref(t), _stream(stream)))
        return m, v, t.value

    def set_state(self, m, v, t: int, stream=None) -> None:
        m = np.ascontiguousarray(m, dtype=np.float64)
        v = np.ascontiguousarray(v, dtype=np.float64)
        if m.size != self.count or v.size != self.count:
            raise ValueError(f"Adam moments need {self.count} values each")
        L.check(self._lib.nnqs_screen_set_state(self.handle, m.ctypes.data_as(ctypes.c_void_p),
                                                v.ctypes.data_as(ctypes.c_void_p), int(t), _stream(stream)))

    def save(self, path: str, stream=None) -> None:
        """Writes the FP64 master weights, the Adam state and the shape to
        ``path`` (a safetensors file: no code runs when it is read back), so
        that training can resume where it stopped."""
        from safetensors.numpy import save_file
        m, v, t = self.state(stream)
        save_file({"weights": self.weights(stream), "adam_m": m, "adam_v": v,
                   "adam_t": np.array([t], dtype=np.int64),
                   "shape": np.array([self.n_spin_orb, self.hidden], dtype=np.int64)}, path)

    @classmethod
    def load(cls, path: str) -> "Screen":
        """A screen with the weights, shape and (when stored) Adam state
        written by :meth:`save`."""
        from safetensors.numpy import load_file
        d = load_file(path)
        n_spin_orb, hidden = (int(v) for v in d["shape"])
        scr = cls(n_spin_orb, hidden, d["weights"])
        if "adam_m" in d:
            scr.set_state(d["adam_m"], d["adam_v"], int(d["adam_t"][0]))
        return scr

    def forward(self, xkeys, exc, precision: int = NNQS_FP64, out=None, stream=None):
        n = xkeys.shape[0]
        _need(xkeys, "xkeys", _KEY_DTYPES, (n, 2))
        _need(exc, "exc", (torch.uint8,), (n, 4))
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=xkeys.device)
        L.check(self._lib.nnqs_screen_forward(self.handle, _ptr(xkeys), _ptr(exc), n, int(precision), _ptr(out),
                                              _stream(stream)))
        return out

    def gradient(self, xkeys, exc, target, precision: int = NNQS_FP64, grad=None, loss=None, stream=None):
        n = xkeys.shape[0]
        _need(xkeys, "xkeys", _KEY_DTYPES, (n, 2))
        _need(exc, "exc", (torch.uint8,), (n, 4))
        _need(target, "target", (torch.float64,), (n,))
        if grad is None:
            grad = torch.empty(self.count, dtype=torch.float64, device=xkeys.device)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float64, device=xkeys.device)
        L.check(self._lib.nnqs_screen_gradient(self.handle, _ptr(xkeys), _ptr(exc), _ptr(target), n, int(precision),
                                               _ptr(grad), _ptr(loss), _stream(stream)))
        return grad, loss

    def judge(self, xkeys, exc, target, precision: int = NNQS_BF16, max_rmse: float = 1.0, stream=None):
        """``(rmse, usable)`` of the fallback judge (``nnqs_screen_judge``)."""
        n = xkeys.shape[0]
        _need(xkeys, "xkeys", _KEY_DTYPES, (n, 2))
        _need(exc, "exc", (torch.uint8,), (n, 4))
        _need(target, "target", (torch.float64,), (n,))
        rmse, ok = ctypes.c_double(), ctypes.c_int32()
        L.check(self._lib.nnqs_screen_judge(self.handle, _ptr(xkeys), _ptr(exc), _ptr(target), n, int(precision),
                                            float(max_rmse), ctypes.byref(rmse), ctypes.byref(ok), _stream(stream)))
        return rmse.value, bool(ok.value)

    def adam_step(self, grad, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        _need(grad, "grad", (torch.float64,), (self.count,))
        L.check(self._lib.nnqs_screen_adam_step(self.handle, _ptr(grad), float(lr), float(beta1), float(beta2),
                                                float(eps), _stream(stream)))

    def close(self):
        if getattr(self, "handle", None):
            self._lib.nnqs_screen_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ------------------------------------------------------------------- Pauli
def pauli_build_host(n_spin_orb: int, h, g, e_core: float = 0.0):
    """Grouped Pauli form of the Hamiltonian, built on the host
    (``nnqs_pauli_build_host``): ``(xy [NK, 2] uint64, idx [NK + 1] int64,
    zm [NT, 2] uint64, coef [NT] float64)``."""
    lib = L.load()
    h = np.ascontiguousarray(h, dtype=np.float64)
    g = np.ascontiguousarray(g, dtype=np.float64)
    nk, nt = ctypes.c_int64(0), ctypes.c_int64(0)
    L.check(lib.nnqs_pauli_build_host(int(n_spin_orb), h.ctypes.data_as(ctypes.c_void_p),
                                      g.ctypes.data_as(ctypes.c_void_p), float(e_core), ctypes.byref(nk),
                                      ctypes.byref(nt), None, None, None, None))
    xy = np.zeros((nk.value, 2), np.uint64)
    idx = np.zeros(nk.value + 1, np.int64)
    zm = np.zeros((nt.value, 2), np.uint64)
    coef = np.zeros(nt.value, np.float64)
    L.check(lib.nnqs_pauli_build_host(int(n_spin_orb), h.ctypes.data_as(ctypes.c_void_p),
                                      g.ctypes.data_as(ctypes.c_void_p), float(e_core), ctypes.byref(nk),
                                      ctypes.byref(nt), xy.ctypes.data_as(ctypes.c_void_p),
                                      idx.ctypes.data_as(ctypes.c_void_p), zm.ctypes.data_as(ctypes.c_void_p),
                                      coef.ctypes.data_as(ctypes.c_void_p)))
    return xy, idx, zm, coef


class Pauli:
    """Grouped Pauli-string Hamiltonian of a system on the device (``nnqs_pauli_*``)."""

    def __init__(self, system: System):
        self._lib = L.load()
        self.system = system
        out = ctypes.c_void_p()
        L.check(self._lib.nnqs_pauli_create(ctypes.byref(out), system.handle))
        self.handle = out

    def info(self) -> dict:
        v = [ctypes.c_int64(0) for _ in range(4)]
        L.check(self._lib.nnqs_pauli_info(self.handle, *[ctypes.byref(x) for x in v]))
        return dict(zip(("groups", "strings", "bytes_grouped", "bytes_flat"), [x.value for x in v]))

    def close(self):
        if getattr(self, "handle", None):
            self._lib.nnqs_pauli_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def eloc_pauli(pauli: Pauli, table: Table, keys, counts, logabs, phase, eloc=None, energy=None,
               with_energy: bool = True, stream=None):
    """Sample-aware local energies over the Pauli groups (``nnqs_eloc_pauli``)."""
    n = keys.shape[0]
    _need(keys, "keys", _KEY_DTYPES, (n, 2))
    _need(logabs, "logabs", (torch.float64,), (n,))
    _need(phase, "phase", (torch.float64,), (n,))
    if with_energy:
        _need(counts, "counts", (torch.int32, torch.uint32), (n,))
        if energy is None:
            energy = torch.empty(4, dtype=torch.float64, device=keys.device)
    if eloc is None:
        eloc = torch.empty((n, 2), dtype=torch.float64, device=keys.device)
    L.check(L.load().nnqs_eloc_pauli(pauli.handle, table.handle, _ptr(keys), _ptr(counts) if with_energy else None,
                                     _ptr(logabs), _ptr(phase), n, _ptr(eloc), _ptr(energy) if with_energy else None,
                                     0, _stream(stream)))
    return eloc, (energy if with_energy else None)


# ------------------------------------------------------------------- batch
class Batch:
    """Many systems in one persistent sample-aware launch (``nnqs_batch_*``).

    ``items`` is a list of dicts with keys ``system``, ``table``, ``keys``,
    ``logabs``, ``phase`` (device tensors; with a ``model`` they are outputs),
    ``eloc`` and optionally ``model``, ``counts``, ``energy``.  The tensors
    must stay alive as long as the batch."""

    def __init__(self, items):
        self._lib = L.load()
        arr = (L.BatchItem * len(items))()
        self._keep = []
        for k, it in enumerate(items):
            n = it["keys"].shape[0]
            _need(it["keys"], "keys", _KEY_DTYPES, (n, 2))
            _need(it["logabs"], "logabs", (torch.float64,), (n,))
            _need(it["phase"], "phase", (torch.float64,), (n,))
            _need(it["eloc"], "eloc", (torch.float64,), (n, 2))
            if it.get("counts") is not None:
                _need(it["counts"], "counts", (torch.int32, torch.uint32), (n,))
            if it.get("energy") is not None:
                _need(it["energy"], "energy", (torch.float64,), (4,))
            model = it.get("model")
            arr[k] = L.BatchItem(it["system"].handle, it["table"].handle, model.handle if model is not None else None,
                                 _ptr(it["keys"]), _ptr(it.get("counts")), _ptr(it["logabs"]), _ptr(it["phase"]), n,
                                 _ptr(it["eloc"]), _ptr(it.get("energy")))
            self._keep.append(it)
        out = ctypes.c_void_p()
        L.check(self._lib.nnqs_batch_create(ctypes.byref(out), arr, len(items)))
        self.handle = out

    def run(self, stream=None):
        L.check(self._lib.nnqs_batch_run(self.handle, _stream(stream)))

    def capture(self, stream):
        L.check(self._lib.nnqs_batch_capture(self.handle, _stream(stream)))

    def launch(self, stream):
        L.check(self._lib.nnqs_batch_launch(self.handle, _stream(stream)))

    def set_tune(self, **kw):
        t = Tune(*[int(kw.get(f, 0)) for f, _ in Tune._fields_])
        L.check(self._lib.nnqs_batch_set_tune(self.handle, ctypes.byref(t)))

    def get_tune(self) -> dict:
        t = Tune()
        L.check(self._lib.nnqs_batch_get_tune(self.handle, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in Tune._fields_}

    def tune_key(self) -> str:
        """Autotuner cache key of the whole batch: the device, the item count
        and a digest of every item's own workload key."""
        keys = [tune_key(it["system"], it["keys"].shape[0]) for it in self._keep]
        digest = hashlib.sha256("|".join(keys).encode()).hexdigest()[:16]
        return f"{keys[0].split(':')[0]}:batch{len(keys)}:{digest}"

    def autotune(self, reps: int = 2, cache_path: str | None = None, stream=None):
        """Times the candidate schedules and keeps the fastest; returns
        ``(tune dict, best step ms)``.  With ``cache_path`` (default: the
        ``NNQS_TUNE_CACHE`` environment variable) a schedule stored there for
        this batch's key is used without timing, and a newly timed one is
        stored (``nnqs_tune_cache_*``)."""
        if cache_path is None:
            cache_path = os.environ.get("NNQS_TUNE_CACHE") or None
        key = self.tune_key() if cache_path is not None else None
        if key is not None:
            hit = tune_cache_lookup(cache_path, key)
            if hit is not None:
                self.set_tune(**hit[0])
                return hit
        t = Tune()
        ms = ctypes.c_double()
        L.check(self._lib.nnqs_batch_autotune(self.handle, int(reps), ctypes.byref(t), ctypes.byref(ms),
                                              _stream(stream)))
        tune = {f: getattr(t, f) for f, _ in Tune._fields_}
        if key is not None:
            tune_cache_store(cache_path, key, tune, ms.value)
        return tune, ms.value

    def close(self):
        if getattr(self, "handle", None):
            self._lib.nnqs_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchModel:
    """Full local energies of many systems in one step (``nnqs_batch_model_*``):
    BF16 network, one persistent launch of the prefix-reusing forward over the
    connections of every item.  ``items``: dicts with ``system``, ``model``,
    ``keys``, ``eloc`` and optionally ``counts``, ``energy`` (device tensors
    that must stay alive as long as the batch)."""

    def __init__(self, items):
        self._lib = L.load()
        arr = (L.BatchModelItem * len(items))()
        self._keep = []
        for k, it in enumerate(items):
            n = it["keys"].shape[0]
            _need(it["keys"], "keys", _KEY_DTYPES, (n, 2))
            _need(it["eloc"], "eloc", (torch.float64,), (n, 2))
            if it.get("counts") is not None:
                _need(it["counts"], "counts", (torch.int32, torch.uint32), (n,))
            if it.get("energy") is not None:
                _need(it["energy"], "energy", (torch.float64,), (4,))
            arr[k] = L.BatchModelItem(it["system"].handle, it["model"].handle, _ptr(it["keys"]),
                                      _ptr(it.get("counts")), n, _ptr(it["eloc"]), _ptr(it.get("energy")))
            self._keep.append(it)
        out = ctypes.c_void_p()
        L.check(self._lib.nnqs_batch_model_create(ctypes.byref(out), arr, len(items)))
        self.handle = out

    def run(self, stream=None):
        L.check(self._lib.nnqs_batch_model_run(self.handle, _stream(stream)))

    def capture(self, stream):
        L.check(self._lib.nnqs_batch_model_capture(self.handle, _stream(stream)))

    def launch(self, stream):
        L.check(self._lib.nnqs_batch_model_launch(self.handle, _stream(stream)))

    def close(self):
        if getattr(self, "handle", None):
            self._lib.nnqs_batch_model_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
