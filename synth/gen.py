"""Seeded generators for integrals, occupation bit strings, amplitudes, counts
and model weights.

Conventions fixed here and used by every consumer:

* ``K`` spatial orbitals, ``N = 2K`` spin orbitals; spin orbital ``p = 2*i + s``
  with ``s = 0`` spin up and ``s = 1`` spin down (the paper maps spatial orbital
  ``i`` to the adjacent qubit pair, up first; Section 3.3, Eq. 12).
* A configuration is a 128-bit key stored as two ``uint64`` words: bit ``p`` of
  the key is the occupation of spin orbital ``p``; word 0 holds bits 0-63 and
  word 1 bits 64-127 (the packed-integer sample table of Section 3.4, item 5).
* Integrals are spatial and in chemists' notation: ``h[i, j]`` and
  ``g[i, j, k, l] = (ij|kl)``, 8-fold symmetric; the core energy is 0.

Seeds are ``numpy.random.default_rng([16705, cfg, sys])``; model weights use
``[16705, cfg, sys, 1]`` so that the sample stream does not depend on them.
"""
from __future__ import annotations

import dataclasses
import itertools
import math

import numpy as np

SEED_ROOT = 16705
_CHUNK = 1 << 16  # fixed draw chunk so that the sample stream is reproducible


# ---------------------------------------------------------------- bit packing
def pack_occupations(occ: np.ndarray) -> np.ndarray:
    """``occ[B, 2, K]`` (spin, spatial) booleans -> ``uint64[B, 2]`` keys."""
    occ = np.asarray(occ, dtype=bool)
    B, two, K = occ.shape
    assert two == 2 and 2 * K <= 128
    keys = np.zeros((B, 2), dtype=np.uint64)
    for i in range(K):
        for s in range(2):
            p = 2 * i + s
            keys[:, p >> 6] |= occ[:, s, i].astype(np.uint64) << np.uint64(p & 63)
    return keys


def unpack_keys(keys: np.ndarray, K: int) -> np.ndarray:
    """Inverse of :func:`pack_occupations`: ``uint64[B, 2]`` -> ``bool[B, 2, K]``."""
    keys = np.asarray(keys, dtype=np.uint64).reshape(-1, 2)
    occ = np.zeros((keys.shape[0], 2, K), dtype=bool)
    for i in range(K):
        for s in range(2):
            p = 2 * i + s
            occ[:, s, i] = ((keys[:, p >> 6] >> np.uint64(p & 63)) & np.uint64(1)) != 0
    return occ


def hf_key(K: int, n_up: int, n_dn: int) -> np.ndarray:
    """Lowest-orbital (Hartree-Fock reference) occupation as a ``uint64[2]`` key."""
    occ = np.zeros((1, 2, K), dtype=bool)
    occ[0, 0, :n_up] = True
    occ[0, 1, :n_dn] = True
    return pack_occupations(occ)[0]


def all_determinants(K: int, n_up: int, n_dn: int) -> np.ndarray:
    """Every configuration of the (n_up, n_dn) sector, up-combination major."""
    rows = []
    for up in itertools.combinations(range(K), n_up):
        for dn in itertools.combinations(range(K), n_dn):
            o = np.zeros((2, K), dtype=bool)
            o[0, list(up)] = True
            o[1, list(dn)] = True
            rows.append(o)
    return pack_occupations(np.stack(rows))


def sector_size(K: int, n_up: int, n_dn: int) -> int:
    return math.comb(K, n_up) * math.comb(K, n_dn)


# ----------------------------------------------------------------- integrals
def integrals(K: int, rng: np.random.Generator, decay: float | None = None,
              n_chol: int = 8, h_std: float = 0.5, l_std: float = 0.3):
    """Random symmetric one-body ``h`` and 8-fold symmetric positive
    semi-definite two-body ``g[p,q,r,s] = sum_l L[l,p,q] L[l,r,s]``.

    ``h = (A + A^T)/2 + diag(linspace(-2, -0.5, K))`` with ``A ~ N(0, h_std)``;
    each ``L[l]`` is a symmetric matrix whose upper triangle is drawn iid from
    ``N(0, l_std)``.  With ``decay`` set, ``A`` and every ``L[l]`` are multiplied
    entrywise by ``exp(-|p-q|/decay)``.
    """
    A = rng.normal(0.0, h_std, size=(K, K))
    Ls = np.empty((n_chol, K, K))
    iu = np.triu_indices(K)
    for l in range(n_chol):
        M = np.zeros((K, K))
        M[iu] = rng.normal(0.0, l_std, size=len(iu[0]))
        Ls[l] = M + np.triu(M, 1).T
    if decay is not None:
        idx = np.arange(K)
        D = np.exp(-np.abs(idx[:, None] - idx[None, :]) / float(decay))
        A = A * D
        Ls = Ls * D[None]
    h = 0.5 * (A + A.T) + np.diag(np.linspace(-2.0, -0.5, K))
    g = np.einsum("lpq,lrs->pqrs", Ls, Ls, optimize=True)
    # exact 8-fold symmetry (the einsum is symmetric up to rounding only)
    g = (g + g.transpose(1, 0, 2, 3)) * 0.5
    g = (g + g.transpose(0, 1, 3, 2)) * 0.5
    g = (g + g.transpose(2, 3, 0, 1)) * 0.5
    return np.ascontiguousarray(h), np.ascontiguousarray(g), 0.0


# ------------------------------------------------------------------- samples
def _popcount64(a: np.ndarray) -> np.ndarray:
    a = a.astype(np.uint64)
    c = np.zeros(a.shape, dtype=np.int64)
    for b in range(64):
        c += ((a >> np.uint64(b)) & np.uint64(1)).astype(np.int64)
    return c


def excitation_level(keys: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """Number of electrons outside the reference: popcount(x & ~ref)."""
    keys = np.asarray(keys, dtype=np.uint64).reshape(-1, 2)
    return _popcount64(keys[:, 0] & ~ref[0]) + _popcount64(keys[:, 1] & ~ref[1])


def geometric_samples(K: int, n_up: int, n_dn: int, n_unique: int,
                      rng: np.random.Generator, p_level: float = 0.4,
                      fermi_decay: float | None = None):
    """Unique configurations drawn around the reference occupation.

    Each draw takes a level ``k`` with ``P(k) = p (1-p)^k`` (k = 0, 1, ...) and
    applies ``k`` random moves; a move picks a spin uniformly, then one occupied
    and one empty orbital of that spin, and moves the electron.  Draws
    continue until ``n_unique`` distinct keys are seen; the first occurrence
    order is kept.  Returns ``(keys uint64[n, 2], level int64[n])``.

    With ``fermi_decay = None`` the two orbitals are uniform.  With a value
    ``lam`` an occupied orbital ``i`` below the Fermi level ``F`` (the
    electron count of that spin) is picked with weight ``exp(-lam (F-1-i))``
    and an empty orbital ``a`` above it with weight ``exp(-lam (a-F))``
    (orbitals on the other side of ``F`` weigh 1), so that samples stay near
    the Fermi level, where a model with an orbital-ordered logit bias puts
    its weight.
    """
    n_sector = sector_size(K, n_up, n_dn)
    if n_unique > n_sector:
        raise ValueError(f"n_unique={n_unique} exceeds the sector size {n_sector}")
    ref = hf_key(K, n_up, n_dn)
    found: list[np.ndarray] = []
    n_found = 0
    seen: set = set()
    stall = 0
    while n_found < n_unique:
        B = _CHUNK
        levels = rng.geometric(p_level, size=B) - 1
        occ = np.zeros((B, 2, K), dtype=bool)
        occ[:, 0, :n_up] = True
        occ[:, 1, :n_dn] = True
        rows = np.arange(B)
        for t in range(int(levels.max())):
            act = levels > t
            spin = rng.integers(0, 2, size=B)
            o = occ[rows, spin]
            r_occ = rng.random((B, K))
            r_emp = rng.random((B, K))
            if fermi_decay is None:
                ri = np.where(o, r_occ, -1.0).argmax(axis=1)
                ra = np.where(~o, r_emp, -1.0).argmax(axis=1)
            else:
                # weighted choice by the Gumbel-max rule: argmax(log w + G)
                F = np.where(spin == 0, n_up, n_dn)[:, None]
                orb = np.arange(K)[None, :]
                lw_hole = -fermi_decay * np.maximum(0, F - 1 - orb)
                lw_part = -fermi_decay * np.maximum(0, orb - F)
                g_occ = -np.log(-np.log(np.maximum(r_occ, 1e-300)))
                g_emp = -np.log(-np.log(np.maximum(r_emp, 1e-300)))
                ri = np.where(o, lw_hole + g_occ, -np.inf).argmax(axis=1)
                ra = np.where(~o, lw_part + g_emp, -np.inf).argmax(axis=1)
            ok = act & o.any(axis=1) & (~o).any(axis=1)
            occ[rows[ok], spin[ok], ri[ok]] = False
            occ[rows[ok], spin[ok], ra[ok]] = True
        keys = pack_occupations(occ)
        before = n_found
        for w0, w1 in zip(keys[:, 0].tolist(), keys[:, 1].tolist()):
            if (w0, w1) in seen:
                continue
            seen.add((w0, w1))
            found.append(np.array([w0, w1], dtype=np.uint64))
            n_found += 1
            if n_found == n_unique:
                break
        stall = stall + 1 if n_found == before else 0
        if stall > 64:
            raise RuntimeError("sample generator stalled; n_unique too close to the sector size")
    keys = np.stack(found[:n_unique]).astype(np.uint64)
    return keys, excitation_level(keys, ref)


def sample_amplitudes(level: np.ndarray, rng: np.random.Generator,
                      slope: float = -1.5, noise: float = 0.3):
    """``log|psi| = slope * level + N(0, noise)``; phase uniform in [0, 2*pi)."""
    n = level.shape[0]
    logabs = slope * level.astype(np.float64) + rng.normal(0.0, noise, size=n)
    phase = rng.uniform(0.0, 2.0 * np.pi, size=n)
    return logabs, phase


def sample_counts(n: int, rng: np.random.Generator, mean: float = 20.0) -> np.ndarray:
    """Occurrence counts ``max(1, Poisson(mean))`` as ``uint32``."""
    return np.maximum(1, rng.poisson(mean, size=n)).astype(np.uint32)


# --------------------------------------------------------------- model weights
@dataclasses.dataclass(frozen=True)
class TransformerShape:
    K: int
    d_model: int = 64
    n_layers: int = 4
    n_heads: int = 4
    d_ff: int = 256
    phase_hidden: int = 512


def transformer_weights(shape: TransformerShape, n_up: int, n_dn: int,
                        rng: np.random.Generator, beta: float = 0.6,
                        std: float = 0.02) -> dict:
    """Random decoder-only transformer (amplitude) and phase MLP weights.

    Matrices are ``[in, out]`` (``y = x @ W + b``), all float32.  ``logit_bias``
    is a fixed, untrained ``[K, 4]`` table ``beta * S(i, t)`` indexed by spatial
    orbital ``i`` and token ``t = n_up(i) + 2 n_dn(i)``, where ``S`` charges
    ``i - F + 1`` for an electron of a spin above that spin's reference level
    ``F = n_spin`` and ``F - i`` for a hole below it.
    """
    K, d, L, dff, P = shape.K, shape.d_model, shape.n_layers, shape.d_ff, shape.phase_hidden
    N = 2 * K
    f32 = np.float32

    def nrm(*s, sd=std):
        return rng.normal(0.0, sd, size=s).astype(f32)

    w = {
        "tok_emb": nrm(5, d),
        "pos_emb": nrm(K, d),
    }
    for l in range(L):
        w[f"l{l}.ln1_g"] = (1.0 + nrm(d)).astype(f32)
        w[f"l{l}.ln1_b"] = nrm(d)
        w[f"l{l}.wq"] = nrm(d, d)
        w[f"l{l}.bq"] = nrm(d)
        w[f"l{l}.wk"] = nrm(d, d)
        w[f"l{l}.bk"] = nrm(d)
        w[f"l{l}.wv"] = nrm(d, d)
        w[f"l{l}.bv"] = nrm(d)
        w[f"l{l}.wo"] = nrm(d, d)
        w[f"l{l}.bo"] = nrm(d)
        w[f"l{l}.ln2_g"] = (1.0 + nrm(d)).astype(f32)
        w[f"l{l}.ln2_b"] = nrm(d)
        w[f"l{l}.w1"] = nrm(d, dff)
        w[f"l{l}.b1"] = nrm(dff)
        w[f"l{l}.w2"] = nrm(dff, d)
        w[f"l{l}.b2"] = nrm(d)
    w["lnf_g"] = (1.0 + nrm(d)).astype(f32)
    w["lnf_b"] = nrm(d)
    w["head_w"] = nrm(d, 4, sd=1.0 / math.sqrt(d))
    w["head_b"] = nrm(4)
    S = np.zeros((K, 4))
    for i in range(K):
        for t in range(4):
            for s, F in ((0, n_up), (1, n_dn)):
                bit = (t >> s) & 1
                if i >= F:
                    S[i, t] -= bit * (i - F + 1)
                else:
                    S[i, t] -= (1 - bit) * (F - i)
    w["logit_bias"] = (beta * S).astype(f32)
    w["ph_w1"] = nrm(N, P, sd=1.0 / math.sqrt(N))
    w["ph_b1"] = nrm(P)
    w["ph_w2"] = nrm(P, P, sd=1.0 / math.sqrt(P))
    w["ph_b2"] = nrm(P)
    w["ph_w3"] = nrm(P, 1, sd=1.0 / math.sqrt(P))
    w["ph_b3"] = nrm(1)
    return w


# ------------------------------------------------------------------- configs
_CONFIGS = {
    # cfg: (K, n_up, n_dn, n_unique or None for the whole sector, decay, model)
    1: (4, 2, 2, None, None, False),
    2: (24, 6, 6, 65536, 8.0, False),
    3: (60, 20, 20, 1_000_000, 8.0, True),
    5: (60, 20, 20, 1_000_000, 8.0, True),
}


def batched_system_specs(n_systems: int = 32):
    """``(K, n_up, n_dn, n_unique)`` for the multi-system batch: ``N`` uniform
    over the even numbers 20..120, ``n = 2*round(N/6)`` split evenly, unique
    sample count log-uniform in [1e3, 1e5], capped at half the sector size."""
    rng = np.random.default_rng([SEED_ROOT, 4])
    Ns = rng.integers(10, 61, size=n_systems) * 2
    nus = np.exp(rng.uniform(np.log(1e3), np.log(1e5), size=n_systems)).round().astype(int)
    specs = []
    for N, nu in zip(Ns.tolist(), nus.tolist()):
        half = int(round(N / 6))
        specs.append((N // 2, half, half, int(min(nu, sector_size(N // 2, half, half) // 2))))
    return specs


def config_inputs(cfg: int, sys: int = 0, *, K: int | None = None, n_up: int | None = None,
                  n_dn: int | None = None, n_unique: int | None = None,
                  decay: float | None = "default", model: bool | None = None,
                  beta: float = 0.6) -> dict:
    """All inputs of one synthetic system.

    ``cfg`` selects the recipe (1: K=4 whole sector; 2: K=24 65,536 samples;
    3/5: K=60 10^6 samples with a model; 4: one system ``sys`` of the batch).
    Keyword overrides give smaller instances of the same recipe for tests.
    """
    if cfg == 4:
        Kd, nu_, nd_, nuq = batched_system_specs()[sys]
        base = (Kd, nu_, nd_, nuq, 8.0, True)
    else:
        base = _CONFIGS[cfg]
    K = base[0] if K is None else K
    n_up = base[1] if n_up is None else n_up
    n_dn = base[2] if n_dn is None else n_dn
    n_unique = base[3] if n_unique is None else n_unique
    decay = base[4] if decay == "default" else decay
    model = base[5] if model is None else model

    rng = np.random.default_rng([SEED_ROOT, cfg, sys])
    h, g, e_core = integrals(K, rng, decay=decay)
    if n_unique is None:
        keys = all_determinants(K, n_up, n_dn)
        level = excitation_level(keys, hf_key(K, n_up, n_dn))
        logabs = rng.normal(0.0, 1.0, size=keys.shape[0])
        phase = rng.uniform(0.0, 2.0 * np.pi, size=keys.shape[0])
        counts = np.ones(keys.shape[0], dtype=np.uint32)
    else:
        # the full-E_loc workloads (3, 5) draw moves near the Fermi level with
        # the decay of the model's own logit bias (|psi|^2 falls by
        # exp(-beta) per orbital); the batch (4) keeps uniform moves
        fermi = beta if (model and cfg in (3, 5)) else None
        keys, level = geometric_samples(K, n_up, n_dn, n_unique, rng, fermi_decay=fermi)
        logabs, phase = sample_amplitudes(level, rng)
        counts = sample_counts(keys.shape[0], rng)
    out = dict(cfg=cfg, sys=sys, K=K, N=2 * K, n_up=n_up, n_dn=n_dn, h=h, g=g, e_core=e_core,
               keys=np.ascontiguousarray(keys), level=level, logabs=logabs, phase=phase,
               counts=counts)
    if model:
        shape = TransformerShape(K=K)
        mrng = np.random.default_rng([SEED_ROOT, cfg, sys, 1])
        out["model_shape"] = shape
        out["weights"] = transformer_weights(shape, n_up, n_dn, mrng, beta=beta)
    return out
