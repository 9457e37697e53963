"""Helpers shared by the GPU tests: device copies of synthetic inputs and the
per-sample tolerance rule for local energies."""
from __future__ import annotations

import numpy as np
import torch


def dev(a, dtype=None):
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.view(np.int64)
    t = torch.from_numpy(a.copy())
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def keys_np(t):
    return t.cpu().numpy().view(np.uint64)


def eloc_complex(t):
    a = t.cpu().numpy()
    return a[:, 0] + 1j * a[:, 1]


def assert_eloc_close(gpu, ora, absum, rel=1e-10, label=""):
    """Per-sample bar: |dE| <= rel |E_ora|; where cancellation leaves
    |E_ora| < 1e-3 A(x), with A = sum |H_xx'| |psi'/psi|, the bar is rel A(x)."""
    gpu = np.asarray(gpu)
    ora = np.asarray(ora)
    d = np.abs(gpu - ora)
    scale = np.where(np.abs(ora) >= 1e-3 * absum, np.abs(ora), absum)
    bad = ~(d <= rel * np.maximum(scale, 1e-300))
    if bad.any():
        k = int(np.flatnonzero(bad)[0])
        raise AssertionError(f"{label}: {int(bad.sum())} samples exceed the bar; first k={k} "
                             f"gpu={gpu[k]} oracle={ora[k]} absum={absum[k]} rel_err={d[k] / scale[k]:.3e}")
    return float(np.max(d / np.maximum(scale, 1e-300)))
