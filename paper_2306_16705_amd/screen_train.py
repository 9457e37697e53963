"""Training driver of the learned screen (argument marshalling around the C ABI).

Training pairs are drawn from the method itself: random connected
configurations x' of given samples (``nnqs_connections``) labelled with the
model's own log|psi(x')| (``nnqs_model_logpsi``).  The screen's forward and
backward passes and the Adam step are the library's kernels
(``nnqs_screen_gradient`` / ``nnqs_screen_adam_step``); this module only picks
minibatches.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import api


def init_weights(n_spin_orb: int, hidden: int, seed: int = 0) -> np.ndarray:
    """Gaussian initial weights, std 1/sqrt(fan_in), zero biases (layout of
    ``nnqs_screen_weight_count``)."""
    N, H = n_spin_orb, hidden
    rng = np.random.default_rng(seed)
    parts = [rng.normal(0.0, 1.0 / math.sqrt(2 * N), size=5 * N * H),  # about 2N inputs are active
             np.zeros(H),
             rng.normal(0.0, 1.0 / math.sqrt(H), size=H * H),
             np.zeros(H),
             rng.normal(0.0, 1.0 / math.sqrt(H), size=H),
             np.zeros(1)]
    return np.concatenate(parts)


def connection_dataset(system: api.System, model: api.Model, keys, per_sample: int, seed: int = 0,
                       precision: int = api.NNQS_BF16, batch_samples: int = 8):
    """``(xkeys [m, 2], exc [m, 4] uint8, label [m] float64)`` device tensors:
    ``per_sample`` uniformly random connections of every sample in ``keys``
    with the model's log|psi(x')| as the label."""
    gen = torch.Generator(device=keys.device)
    gen.manual_seed(seed)
    C = system.connection_count
    xs, es = [], []
    for b0 in range(0, keys.shape[0], batch_samples):
        kb = keys[b0:b0 + batch_samples]
        out = api.connections(system, kb)
        idx = torch.randint(0, C, (kb.shape[0], per_sample), generator=gen, device=keys.device)
        xs.append(torch.gather(out["xprime"], 1, idx[..., None].expand(-1, -1, 2)).reshape(-1, 2))
        es.append(torch.gather(out["exc"], 1, idx[..., None].expand(-1, -1, 4)).reshape(-1, 4))
        del out
    xkeys = torch.cat(xs).contiguous()
    exc = torch.cat(es).contiguous()
    label, _ = api.model_logpsi(model, xkeys, precision)
    return xkeys, exc, label


def train(screen: api.Screen, xkeys, exc, target, steps: int, batch: int = 4096, lr: float = 1e-3,
          precision: int = api.NNQS_FP32, seed: int = 0, lr_decay_to: float = 0.1):
    """Minibatch Adam on the mean squared error; returns the loss per step
    (host list, read once at the end).  The learning rate decays
    geometrically to ``lr_decay_to * lr`` over the run."""
    gen = torch.Generator(device=xkeys.device)
    gen.manual_seed(seed)
    m = xkeys.shape[0]
    grad = torch.empty(screen.count, dtype=torch.float64, device=xkeys.device)
    losses = torch.empty(steps, dtype=torch.float64, device=xkeys.device)
    decay = lr_decay_to ** (1.0 / max(1, steps - 1))
    for s in range(steps):
        idx = torch.randint(0, m, (min(batch, m),), generator=gen, device=xkeys.device)
        screen.gradient(xkeys[idx].contiguous(), exc[idx].contiguous(), target[idx].contiguous(), precision,
                        grad=grad, loss=losses[s:s + 1])
        screen.adam_step(grad, lr=lr * decay ** s)
    return losses.cpu().numpy().tolist()


def split(xkeys, exc, target, held_out: float = 0.05, seed: int = 0):
    """Random split of a pair set into (train, held-out) triples."""
    gen = torch.Generator(device=xkeys.device)
    gen.manual_seed(seed)
    perm = torch.randperm(xkeys.shape[0], generator=gen, device=xkeys.device)
    m = max(1, int(round(held_out * xkeys.shape[0])))
    ho, tr = perm[:m], perm[m:]
    return ((xkeys[tr].contiguous(), exc[tr].contiguous(), target[tr].contiguous()),
            (xkeys[ho].contiguous(), exc[ho].contiguous(), target[ho].contiguous()))


def screen_or_plain(screen: api.Screen, xkeys, exc, target, max_rmse: float = 1.0):
    """The screen if its held-out RMSE (the library's fallback judge, in the
    precision the full evaluation uses) is at most ``max_rmse`` nats, else
    ``None`` (the caller then runs the plain evaluation).  Returns
    ``(screen or None, rmse)``."""
    rmse, ok = screen.judge(xkeys, exc, target, api.NNQS_BF16, max_rmse)
    return (screen if ok else None), rmse
