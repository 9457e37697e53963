"""FP64 oracle of the VMC gradient step (test infrastructure only).

* ``logpsi_vjp``: the weighted sum of parameter gradients
  ``sum_b c_b grad log|psi(x_b)| + e_b grad phi(x_b)`` of the ansatz of
  Section 3.1 (Eq. 11, Fig. 2, the Eq. 12 mask, the phase MLP of Section 4.1).
  The forward is written out here in plain float64 PyTorch operations (matrix
  products, an explicit LayerNorm, an explicit causal softmax, erf GELU, a
  masked log-softmax) and the gradient is PyTorch's reverse-mode derivative of
  that forward: the plain definition of the derivative, no hand-written
  backward.
* ``vmc_gradient``: Eq. 7, ``2 Re E_p[(E_loc - E_p[E_loc]) grad ln psi*]`` with
  the sample weights of Eq. 6 (counts over their sum).  With
  ``ln psi = log|psi| + i phi`` the real part splits into
  ``Re(dE) grad log|psi| + Im(dE) grad phi``.
* ``lr_schedule``: Eq. 13 (Section 4.1), the warm-up learning rate.
* ``adamw_step``: AdamW (decoupled weight decay, Loshchilov and Hutter,
  ICLR 2019), the optimizer Section 4.1 names.

The logit-bias table is a fixed part of the ansatz, not a parameter: its
gradient is zero and AdamW leaves it unchanged.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may use
this module.  It shares no code with the HIP library.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from .oracle import net_order

FIXED = ("logit_bias",)


def _tokens(keys: np.ndarray, K: int):
    """Occupation bits [B, 2K] (spin orbital p = 2 i + s) and the token of
    every position [B, K] (position s holds spatial orbital K-1-s; token
    t = n_up(i) + 2 n_dn(i))."""
    keys = np.ascontiguousarray(keys, dtype=np.uint64).reshape(-1, 2)
    B = keys.shape[0]
    bits = np.zeros((B, 2 * K), np.int64)
    for p in range(2 * K):
        word, b = divmod(p, 64)
        bits[:, p] = ((keys[:, word] >> np.uint64(b)) & np.uint64(1)).astype(np.int64)
    orb_tok = bits[:, 0::2] + 2 * bits[:, 1::2]       # token of orbital i
    seq = orb_tok[:, ::-1].copy()                     # token of position s
    return torch.tensor(bits, dtype=torch.float64), torch.tensor(seq)


def _layer_norm(x, g, b):
    mu = x.mean(-1, keepdim=True)
    var = ((x - mu) ** 2).mean(-1, keepdim=True)
    return (x - mu) / torch.sqrt(var + 1e-5) * g + b


def _gelu(x):
    return 0.5 * x * (1.0 + torch.erf(x / math.sqrt(2.0)))


def forward(T: dict, shape, n_up: int, n_dn: int, keys: np.ndarray):
    """(log|psi|, phase) of every key as float64 tensors with autograd
    history; ``T`` maps the weight names to float64 tensors."""
    K, d, L, H = shape.K, shape.d_model, shape.n_layers, shape.n_heads
    dh = d // H
    bits, seq = _tokens(keys, K)
    B = seq.shape[0]
    prev = torch.cat([torch.full((B, 1), 4, dtype=torch.long), seq[:, :-1]], dim=1)
    h = T["tok_emb"][prev] + T["pos_emb"][None]
    causal = torch.tril(torch.ones(K, K, dtype=torch.bool))
    for l in range(L):
        p = lambda k: T[f"l{l}.{k}"]  # noqa: E731
        a = _layer_norm(h, p("ln1_g"), p("ln1_b"))
        heads = []
        for hh in range(H):
            cs = slice(hh * dh, (hh + 1) * dh)
            q = a @ p("wq")[:, cs] + p("bq")[cs]
            k = a @ p("wk")[:, cs] + p("bk")[cs]
            v = a @ p("wv")[:, cs] + p("bv")[cs]
            s = (q @ k.transpose(1, 2)) / math.sqrt(dh)
            s = s.masked_fill(~causal, float("-inf"))
            heads.append(torch.softmax(s, dim=-1) @ v)
        o = torch.cat(heads, dim=-1)
        h = h + o @ p("wo") + p("bo")
        a2 = _layer_norm(h, p("ln2_g"), p("ln2_b"))
        h = h + _gelu(a2 @ p("w1") + p("b1")) @ p("w2") + p("b2")
    af = _layer_norm(h, T["lnf_g"], T["lnf_b"])
    orb = K - 1 - torch.arange(K)
    z = af @ T["head_w"] + T["head_b"] + T["logit_bias"][orb][None]
    # Eq. 12 mask (with the lower bound): token t at position s is allowed if
    # neither spin exceeds its count and the remaining positions can still
    # hold the electrons left to place.
    up, dn = seq & 1, seq >> 1
    ub = (torch.cumsum(up, 1) - up)[..., None]
    db = (torch.cumsum(dn, 1) - dn)[..., None]
    t = torch.arange(4)
    tu, td = (t & 1)[None, None], (t >> 1)[None, None]
    rem = (K - 1 - torch.arange(K))[None, :, None]
    ok = (ub + tu <= n_up) & (db + td <= n_dn) & (n_up - ub - tu <= rem) & (n_dn - db - td <= rem)
    logp = torch.log_softmax(z.masked_fill(~ok, float("-inf")), dim=-1)
    logabs = 0.5 * logp.gather(2, seq[..., None]).squeeze(-1).sum(1)
    z1 = _gelu(bits @ T["ph_w1"] + T["ph_b1"])
    z2 = _gelu(z1 @ T["ph_w2"] + T["ph_b2"])
    phase = (z2 @ T["ph_w3"] + T["ph_b3"]).squeeze(-1)
    return logabs, phase


def _tensors(weights: dict, grad: bool):
    return {k: torch.tensor(np.asarray(v, dtype=np.float64), requires_grad=grad and k not in FIXED)
            for k, v in weights.items()}


def logpsi(weights: dict, shape, n_up: int, n_dn: int, keys):
    """(log|psi|, phase) as float64 numpy arrays."""
    with torch.no_grad():
        la, ph = forward(_tensors(weights, False), shape, n_up, n_dn, keys)
    return la.numpy(), ph.numpy()


def logpsi_vjp(weights: dict, shape, n_up: int, n_dn: int, keys, c_logabs, c_phase) -> dict:
    """sum_b c_logabs[b] grad log|psi_b| + c_phase[b] grad phi_b, per weight
    name (float64 arrays of the weights' shapes; zero for the fixed table)."""
    T = _tensors(weights, True)
    la, ph = forward(T, shape, n_up, n_dn, keys)
    cl = torch.tensor(np.asarray(c_logabs, dtype=np.float64))
    cp = torch.tensor(np.asarray(c_phase, dtype=np.float64))
    (cl @ la + cp @ ph).backward()
    return {k: (t.grad.numpy().copy() if t.grad is not None else np.zeros(t.shape)) for k, t in T.items()}


def vmc_coefficients(weights_b, eloc):
    """Eq. 7 as cotangents: with p_b = w_b / sum w and E = sum_b p_b E_loc(b),
    c_b = 2 p_b Re(E_loc(b) - E) for log|psi| and e_b = 2 p_b Im(E_loc(b) - E)
    for the phase; also returns E."""
    w = np.asarray(weights_b, dtype=np.float64)
    p = w / w.sum()
    e = np.asarray(eloc, dtype=np.complex128)
    E = np.sum(p * e)
    de = e - E
    return 2.0 * p * de.real, 2.0 * p * de.imag, E


def vmc_gradient(weights: dict, shape, n_up: int, n_dn: int, keys, counts, eloc):
    """Eq. 7 gradient (per weight name) and the weighted mean energy."""
    cl, cp, E = vmc_coefficients(counts, eloc)
    return logpsi_vjp(weights, shape, n_up, n_dn, keys, cl, cp), E


def pack(grads: dict, shape) -> np.ndarray:
    """Flatten per-name arrays in the weight layout order."""
    return np.concatenate([np.asarray(grads[k], dtype=np.float64).ravel() for k in net_order(shape.n_layers)])


def unpack(flat: np.ndarray, like: dict, shape) -> dict:
    out, at = {}, 0
    for k in net_order(shape.n_layers):
        n = int(np.asarray(like[k]).size)
        out[k] = np.asarray(flat[at:at + n], dtype=np.float64).reshape(np.asarray(like[k]).shape)
        at += n
    assert at == flat.size
    return out


def fixed_mask(like: dict, shape) -> np.ndarray:
    """1.0 for trainable entries of the flat layout, 0.0 for the fixed table."""
    return np.concatenate([np.full(np.asarray(like[k]).size, 0.0 if k in FIXED else 1.0)
                           for k in net_order(shape.n_layers)])


def lr_schedule(i: int, d_model: int, warmup: int = 4000) -> float:
    """Eq. 13: d_model^-1/2 min(i^-1/2, i warmup^-3/2), iterations from 1."""
    return d_model ** -0.5 * min(i ** -0.5, i * warmup ** -1.5)


def adamw_step(w, g, m, v, t: int, lr: float, beta1: float, beta2: float, eps: float, weight_decay: float,
               trainable=None):
    """One AdamW update (step t >= 1) of flat float64 arrays, returned as new
    arrays (w, m, v): w <- w - lr wd w, then the Adam step with bias-corrected
    moments m / (1 - beta1^t) and v / (1 - beta2^t).  Entries with
    trainable == 0 are left as they are."""
    w = np.asarray(w, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    nw = w * (1.0 - lr * weight_decay) - lr * mh / (np.sqrt(vh) + eps)
    if trainable is not None:
        keep = np.asarray(trainable) == 0
        nw = np.where(keep, w, nw)
        m = np.where(keep, 0.0, m)
        v = np.where(keep, 0.0, v)
    return nw, m, v
