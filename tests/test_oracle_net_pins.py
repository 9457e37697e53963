"""Pins of the FP64 network oracle (amplitude transformer + phase MLP).

* autoregressive normalisation: sum over the sector of |psi|^2 = 1 (Eq. 8 with
  the Eq. 12 mask renormalised, in its lower-bound reading);
* causality: conditionals at a position depend only on earlier tokens;
* an independent PyTorch FP64 implementation built from library routines
  (layer_norm, scaled_dot_product_attention with a causal mask, exact GELU,
  log_softmax) must agree to 1e-12.
"""
import itertools

import numpy as np
import pytest
import torch
import torch.nn.functional as F

import oracle
import synth


def _model(K, nu, nd, seed=3, beta=0.6):
    shape = synth.TransformerShape(K=K)
    rng = np.random.default_rng([synth.SEED_ROOT, 901, seed])
    return shape, synth.transformer_weights(shape, nu, nd, rng, beta=beta)


def torch_logpsi(w, shape, nu, nd, keys):
    """Library-routine reference of the same network, float64 on the CPU."""
    K, d, L, H = shape.K, shape.d_model, shape.n_layers, shape.n_heads
    T = {k: torch.tensor(np.asarray(v, dtype=np.float64)) for k, v in w.items()}
    occ = synth.unpack_keys(keys, K).astype(np.int64)          # [B, 2, K]
    tok_orb = occ[:, 0, :] + 2 * occ[:, 1, :]                  # token per orbital
    seq = torch.tensor(tok_orb[:, ::-1].copy())                # position s <-> orbital K-1-s
    B = seq.shape[0]
    prev = torch.cat([torch.full((B, 1), 4, dtype=torch.long), seq[:, :-1]], dim=1)
    h = T["tok_emb"][prev] + T["pos_emb"][None]
    for l in range(L):
        p = lambda k: T[f"l{l}.{k}"]  # noqa: E731
        a = F.layer_norm(h, (d,), p("ln1_g"), p("ln1_b"), eps=1e-5)
        q = (a @ p("wq") + p("bq")).view(B, K, H, d // H).transpose(1, 2)
        k = (a @ p("wk") + p("bk")).view(B, K, H, d // H).transpose(1, 2)
        v = (a @ p("wv") + p("bv")).view(B, K, H, d // H).transpose(1, 2)
        o = F.scaled_dot_product_attention(q, k, v, is_causal=True).transpose(1, 2).reshape(B, K, d)
        h = h + o @ p("wo") + p("bo")
        a2 = F.layer_norm(h, (d,), p("ln2_g"), p("ln2_b"), eps=1e-5)
        h = h + F.gelu(a2 @ p("w1") + p("b1")) @ p("w2") + p("b2")
    z = F.layer_norm(h, (d,), T["lnf_g"], T["lnf_b"], eps=1e-5) @ T["head_w"] + T["head_b"]
    z = z + T["logit_bias"].flip(0)[None]                      # bias of orbital K-1-s at position s
    up = seq & 1
    dn = seq >> 1
    up_before = torch.cumsum(up, 1) - up
    dn_before = torch.cumsum(dn, 1) - dn
    rem = (K - 1 - torch.arange(K))[None, :, None]
    t = torch.arange(4)
    tu, td = (t & 1)[None, None], (t >> 1)[None, None]
    ub, db = up_before[..., None], dn_before[..., None]
    allowed = (ub + tu <= nu) & (db + td <= nd) & (nu - ub - tu <= rem) & (nd - db - td <= rem)
    logp = torch.log_softmax(z.masked_fill(~allowed, float("-inf")), dim=-1)
    la = 0.5 * logp.gather(2, seq[..., None]).squeeze(-1).sum(1)
    bits = torch.zeros(B, 2 * K, dtype=torch.float64)
    bits[:, 0::2] = torch.tensor(occ[:, 0, :], dtype=torch.float64)
    bits[:, 1::2] = torch.tensor(occ[:, 1, :], dtype=torch.float64)
    z1 = F.gelu(bits @ T["ph_w1"] + T["ph_b1"])
    z2 = F.gelu(z1 @ T["ph_w2"] + T["ph_b2"])
    ph = (z2 @ T["ph_w3"] + T["ph_b3"]).squeeze(-1)
    return la.numpy(), ph.numpy(), logp.numpy()


@pytest.mark.parametrize("K,nu,nd", [(4, 2, 2), (5, 2, 1), (5, 3, 2), (6, 1, 3), (6, 3, 3)])
def test_autoregressive_normalisation(K, nu, nd):
    shape, w = _model(K, nu, nd, beta=0.3)
    keys = synth.all_determinants(K, nu, nd)
    la, _ = oracle.net_logpsi(w, shape, nu, nd, keys)
    assert abs(np.sum(np.exp(2 * la)) - 1.0) < 1e-12


def test_causality():
    K, nu, nd = 8, 3, 3
    shape, w = _model(K, nu, nd)
    keys = synth.all_determinants(K, nu, nd)
    occ = synth.unpack_keys(keys, K)
    tok = (occ[:, 0] + 2 * occ[:, 1])[:, ::-1]       # tokens in autoregressive order
    rng = np.random.default_rng(2)
    for _ in range(20):
        a, b = rng.choice(len(keys), 2, replace=False)
        common = 0
        while common < K and tok[a, common] == tok[b, common]:
            common += 1
        ca = oracle.net_conditionals(w, shape, nu, nd, keys[a])
        cb = oracle.net_conditionals(w, shape, nu, nd, keys[b])
        # positions 0..common depend only on the shared prefix
        assert np.array_equal(ca[: common + 1], cb[: common + 1])
        if common + 1 < K:
            assert not np.array_equal(ca[common + 1:], cb[common + 1:])


def test_mask_and_conditionals_are_distributions():
    K, nu, nd = 6, 2, 3
    shape, w = _model(K, nu, nd)
    for x in synth.all_determinants(K, nu, nd)[::7]:
        c = oracle.net_conditionals(w, shape, nu, nd, x)
        assert np.allclose(np.exp(c).sum(1), 1.0, atol=1e-13)
        assert np.isinf(c).any()  # the mask removes something somewhere


@pytest.mark.parametrize("K,nu,nd,take", [(8, 3, 3, 40), (12, 4, 3, 30), (60, 20, 20, 6)])
def test_matches_library_reference(K, nu, nd, take):
    shape, w = _model(K, nu, nd)
    if K <= 8:
        keys = synth.all_determinants(K, nu, nd)[:take]
    else:
        keys, _ = synth.geometric_samples(K, nu, nd, take, np.random.default_rng(7))
    la, ph = oracle.net_logpsi(w, shape, nu, nd, keys)
    rla, rph, rlogp = torch_logpsi(w, shape, nu, nd, keys)
    assert np.max(np.abs(la - rla)) < 1e-12 * max(1.0, np.abs(rla).max())
    assert np.max(np.abs(ph - rph)) < 1e-12
    c = oracle.net_conditionals(w, shape, nu, nd, keys[0])
    fin = np.isfinite(rlogp[0])
    assert np.array_equal(np.isfinite(c), fin)
    assert np.max(np.abs(c[fin] - rlogp[0][fin])) < 1e-12


def test_full_eloc_equals_table_eloc_over_whole_sector():
    """With every configuration of the sector in the table and the table's
    amplitudes taken from the networks, the sample-aware and the full local
    energies coincide (Section 3.4 item 4 restricts a sum that is complete)."""
    K, nu, nd = 5, 2, 2
    d = synth.config_inputs(1, K=K, n_up=nu, n_dn=nd, model=True)
    shape, w = d["model_shape"], d["weights"]
    keys = d["keys"]
    la, ph = oracle.net_logpsi(w, shape, nu, nd, keys)
    full = oracle.eloc_model(K, nu, nd, d["h"], d["g"], d["e_core"], w, shape, keys)
    tab = oracle.eloc_table(K, nu, nd, d["h"], d["g"], d["e_core"], keys, la, ph, keys, la, ph)
    assert np.max(np.abs(full - tab)) < 1e-11 * max(1.0, np.abs(tab).max())
