"""GPU parity of the network forward and of the full local energy against
the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import assert_eloc_close, dev, eloc_complex

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nn():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_16705_amd as nn
    return nn


def _print_case(name, **kw):
    print(f"[case] {name} {kw}", flush=True)


def _random_connected(d, n_samples, per_sample, seed):
    """Random connected configurations x' of the first samples (oracle enumeration)."""
    rng = np.random.default_rng(seed)
    out = []
    for k in range(n_samples):
        xp, _, _, _ = oracle.connections(d["K"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"], d["keys"][k])
        out.append(xp[rng.choice(len(xp), size=min(per_sample, len(xp)), replace=False)])
    return np.concatenate(out)


@pytest.mark.parametrize("kw", [dict(cfg=1, model=True), dict(cfg=2, K=12, n_up=4, n_dn=3, n_unique=200, model=True),
                                dict(cfg=3, n_unique=8),
                                # the largest sequence (64 positions, no padding rows, two-word keys)
                                dict(cfg=2, K=64, n_up=8, n_dn=8, n_unique=40, model=True),
                                # more configurations than one FP64 pass takes (4,096), ragged tail
                                dict(cfg=2, K=16, n_up=3, n_dn=5, n_unique=5000, model=True)])
def test_logpsi_fp64_matches_oracle(nn, kw):
    kw = dict(kw)
    cfg = kw.pop("cfg")
    d = synth.config_inputs(cfg, **kw)
    _print_case("logpsi_fp64", K=d["K"])
    shape, w = d["model_shape"], d["weights"]
    M = nn.Model(shape, d["n_up"], d["n_dn"], w)
    keys = d["keys"] if d["K"] < 60 else np.concatenate([d["keys"], _random_connected(d, 2, 300, 5)])
    la, ph = nn.model_logpsi(M, dev(keys), nn.NNQS_FP64)
    torch.cuda.synchronize()
    ola, oph = oracle.net_logpsi(w, shape, d["n_up"], d["n_dn"], keys, nthreads=0)
    la, ph = la.cpu().numpy(), ph.cpu().numpy()
    assert np.max(np.abs(la - ola) / np.maximum(1.0, np.abs(ola))) < 1e-12
    assert np.max(np.abs(ph - oph)) < 1e-12


@pytest.mark.parametrize("F", [128, 320])
def test_logpsi_fp64_other_ffn_widths_match_oracle(nn, F):
    """The layer-batched FP64 forward at FFN widths other than 256 (its FFN
    output product then takes the run-time inner dimension and a separate
    LayerNorm statistics pass); larger weights (std 0.2) so that LayerNorm and
    GELU act far from their linear ranges."""
    K, nu, nd = 12, 4, 3
    shape = synth.TransformerShape(K=K, d_model=64, n_layers=2, n_heads=4, d_ff=F, phase_hidden=96)
    w = synth.transformer_weights(shape, nu, nd, np.random.default_rng([synth.SEED_ROOT, 903, F]), std=0.2)
    w = {k: np.asarray(v, dtype=np.float64) for k, v in w.items()}
    keys, _ = synth.geometric_samples(K, nu, nd, 300, np.random.default_rng(7))
    _print_case("logpsi_fp64_ffn", K=K, F=F)
    M = nn.Model(shape, nu, nd, w)
    la, ph = nn.model_logpsi(M, dev(keys), nn.NNQS_FP64)
    torch.cuda.synchronize()
    ola, oph = oracle.net_logpsi(w, shape, nu, nd, keys, nthreads=0)
    la, ph = la.cpu().numpy(), ph.cpu().numpy()
    assert np.max(np.abs(la - ola) / np.maximum(1.0, np.abs(ola))) < 1e-12
    assert np.max(np.abs(ph - oph)) < 1e-12


@pytest.mark.parametrize("kw,take", [(dict(K=5, n_up=2, n_dn=2), None), (dict(K=6, n_up=2, n_dn=3), None),
                                     (dict(K=16, n_up=4, n_dn=4, n_unique=64), 4)])
def test_eloc_model_fp64_matches_oracle(nn, kw, take):
    cfg = 1 if "n_unique" not in kw else 2
    d = synth.config_inputs(cfg, model=True, **kw)
    _print_case("eloc_model_fp64", **kw)
    shape, w = d["model_shape"], d["weights"]
    S = nn.System(d["N"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"])
    M = nn.Model(shape, d["n_up"], d["n_dn"], w)
    keys = d["keys"] if take is None else d["keys"][:take]
    counts = d["counts"][: len(keys)]
    e, en, st = nn.eloc_model(S, M, dev(keys), dev(counts, torch.int32), nn.NNQS_FP64, with_stats=True)
    g = eloc_complex(e)
    ora, absum = oracle.eloc_model(d["K"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"], w, shape, keys,
                                   with_absum=True)
    assert_eloc_close(g, ora, absum, label=str(kw))
    assert st["connections"] == len(keys) * S.connection_count
    ref = oracle.energy(counts, g)
    assert abs(en[0].item() - ref[0]) <= 1e-12 * abs(ref[0])


def test_eloc_model_whole_sector_equals_table_path(nn):
    """Over a whole sector, the full path equals the sample-aware path fed with
    the network's own amplitudes (both on the GPU)."""
    d = synth.config_inputs(1, K=6, n_up=3, n_dn=2, model=True)
    _print_case("eloc_model_vs_table")
    S = nn.System(d["N"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"])
    M = nn.Model(d["model_shape"], d["n_up"], d["n_dn"], d["weights"])
    keys = dev(d["keys"])
    cnt = dev(d["counts"], torch.int32)
    la, ph = nn.model_logpsi(M, keys, nn.NNQS_FP64)
    T = nn.Table(S, capacity=keys.shape[0]).build(keys, la, ph, validate=True)
    e1, _ = nn.eloc_table(S, T, keys, cnt, la, ph)
    e2, _, _ = nn.eloc_model(S, M, keys, cnt, nn.NNQS_FP64)
    torch.cuda.synchronize()
    a, b = eloc_complex(e1), eloc_complex(e2)
    assert np.max(np.abs(a - b)) <= 1e-11 * max(1.0, np.abs(a).max())


@pytest.mark.parametrize("kw", [dict(cfg=1, model=True), dict(cfg=3, n_unique=16),
                                dict(cfg=2, K=64, n_up=8, n_dn=8, n_unique=64, model=True),
                                dict(cfg=2, K=16, n_up=3, n_dn=5, n_unique=37, model=True)])
def test_logpsi_bf16_error_vs_oracle(nn, kw):
    """BF16 MFMA forward: the error against the FP64 oracle is measured and
    bounded (|d log|psi|| <= 0.02 + 1e-3 |log|psi||, |d phase| <= 0.02)."""
    kw = dict(kw)
    cfg = kw.pop("cfg")
    d = synth.config_inputs(cfg, **kw)
    _print_case("logpsi_bf16", K=d["K"])
    shape, w = d["model_shape"], d["weights"]
    M = nn.Model(shape, d["n_up"], d["n_dn"], w)
    keys = d["keys"] if d["K"] < 60 else np.concatenate([d["keys"], _random_connected(d, 2, 500, 9)])
    la, ph = nn.model_logpsi(M, dev(keys), nn.NNQS_BF16)
    torch.cuda.synchronize()
    ola, oph = oracle.net_logpsi(w, shape, d["n_up"], d["n_dn"], keys)
    la, ph = la.cpu().numpy(), ph.cpu().numpy()
    dla, dph = np.abs(la - ola), np.abs(ph - oph)
    print(f"BF16 vs FP64 oracle K={d['K']}: max |dlogabs| {dla.max():.3e} (rel {np.max(dla / np.abs(ola)):.3e}), "
          f"max |dphase| {dph.max():.3e}, n={len(keys)}")
    assert np.all(dla <= 0.02 + 1e-3 * np.abs(ola))
    assert np.all(dph <= 0.02)


@pytest.mark.parametrize("cfg,kw", [(1, dict(K=6, n_up=2, n_dn=3, model=True)),
                                    (2, dict(K=40, n_up=3, n_dn=3, n_unique=3, model=True)),
                                    (2, dict(K=48, n_up=3, n_dn=2, n_unique=2, model=True)),
                                    (2, dict(K=64, n_up=4, n_dn=4, n_unique=2, model=True)),
                                    (3, dict(n_unique=2))])
def test_eloc_model_refined_bf16_equals_fp64_when_all_terms_refined(nn, cfg, kw):
    """Precision ladder: with a refinement threshold far below every term
    (exp(-60) Ha), the BF16 pass only decides what to refine, every term and
    the samples' own amplitudes come from the FP64 network, and the result is
    the FP64 path's.  The refinement evaluates each x' from its first changed
    position on (the diagonal: its last row only), with the sample's FP64
    keys and values below it, so batches pack rows of every length:
    K = 40, 48, 60 and 64 put starts in every 16-row attention block and
    ragged last blocks (K = 40, 60)."""
    d = synth.config_inputs(cfg, **kw)
    _print_case("eloc_model_refine_all", K=d["K"])
    S = nn.System(d["N"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"])
    M = nn.Model(d["model_shape"], d["n_up"], d["n_dn"], d["weights"])
    keys, cnt = dev(d["keys"]), dev(d["counts"], torch.int32)
    e64, en64, _ = nn.eloc_model(S, M, keys, cnt, nn.NNQS_FP64)
    e, en, st = nn.eloc_model(S, M, keys, cnt, nn.NNQS_BF16, refine_nats=60.0, with_stats=True)
    torch.cuda.synchronize()
    a, b = eloc_complex(e64), eloc_complex(e)
    assert st["evaluated"] == st["connections"]
    assert 0 < st["refined"] <= st["connections"]
    assert np.max(np.abs(a - b)) <= 1e-12 * max(1.0, np.abs(a).max())


def test_eloc_model_refinement_shrinks_bf16_error(nn):
    """Precision ladder on N=32 (4 + 4 electrons): the error of the BF16
    path against the FP64 path is stated, and refining every term above
    exp(-8) Ha in FP64 cuts it at least tenfold while re-evaluating only part
    of the connections."""
    d = synth.config_inputs(2, K=16, n_up=4, n_dn=4, n_unique=12, model=True)
    _print_case("eloc_model_refine_error")
    S = nn.System(d["N"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"])
    M = nn.Model(d["model_shape"], d["n_up"], d["n_dn"], d["weights"])
    keys, cnt = dev(d["keys"]), dev(d["counts"], torch.int32)
    e64, en64, _ = nn.eloc_model(S, M, keys, cnt, nn.NNQS_FP64)
    e16, en16, _ = nn.eloc_model(S, M, keys, cnt, nn.NNQS_BF16)
    er, enr, st = nn.eloc_model(S, M, keys, cnt, nn.NNQS_BF16, refine_nats=8.0, with_stats=True)
    torch.cuda.synchronize()
    ref = eloc_complex(e64)
    d16 = np.abs(eloc_complex(e16) - ref)
    dr = np.abs(eloc_complex(er) - ref)
    frac = st["refined"] / st["connections"]
    print(f"E_loc vs FP64: BF16 max {d16.max():.3e} Ha, BF16 + refine(8) max {dr.max():.3e} Ha "
          f"(refined {frac:.3f} of connections); energy {en16[0].item() - en64[0].item():.3e} / "
          f"{enr[0].item() - en64[0].item():.3e} Ha")
    assert dr.max() <= 0.1 * d16.max()
    assert frac < 1.0


@pytest.mark.parametrize("prec", ["bf16", "fp8"])
@pytest.mark.parametrize("kw,take", [(dict(cfg=2, K=16, n_up=4, n_dn=4, n_unique=20, model=True), 6),
                                     (dict(cfg=2, K=64, n_up=8, n_dn=8, n_unique=4, model=True), 1),
                                     (dict(cfg=3, n_unique=2), 1)])
def test_bf16_prefix_reuse_equals_whole_forward(nn, kw, take, prec):
    """The BF16 full path evaluates each x' from its first changed position on,
    with the sample's cached keys and values for the rows before; by causality
    that is the same computation as the whole forward of x'.  E_loc from
    nnqs_eloc_model must equal E_loc assembled from the whole-sequence BF16
    amplitudes of every x' (nnqs_model_logpsi) and the exact matrix elements
    (nnqs_connections), up to FP64 summation order: a difference of one FP32
    rounding in any log|psi(x')| would show at ~1e-8."""
    kw = dict(kw)
    cfg = kw.pop("cfg")
    d = synth.config_inputs(cfg, **kw)
    P = nn.NNQS_BF16 if prec == "bf16" else nn.NNQS_FP8
    _print_case("prefix_vs_whole", K=d["K"], take=take, prec=prec)
    S = nn.System(d["N"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"])
    M = nn.Model(d["model_shape"], d["n_up"], d["n_dn"], d["weights"])
    keys = dev(d["keys"][:take])
    cnt = dev(d["counts"][:take], torch.int32)
    e, _, st = nn.eloc_model(S, M, keys, cnt, P, with_stats=True)
    con = nn.connections(S, keys)
    C = S.connection_count
    xla, xph = nn.model_logpsi(M, con["xprime"].reshape(-1, 2), P)
    sla, sph = nn.model_logpsi(M, keys, P)
    torch.cuda.synchronize()
    hv = con["hxx"].cpu().numpy()
    xla, xph = xla.cpu().numpy().reshape(take, C), xph.cpu().numpy().reshape(take, C)
    sla, sph = sla.cpu().numpy(), sph.cpu().numpy()
    terms = hv * np.exp(xla - sla[:, None]) * np.exp(1j * (xph - sph[:, None]))
    ref = terms.sum(axis=1)
    absum = np.abs(terms).sum(axis=1)
    g = eloc_complex(e)
    assert st["evaluated"] == take * C
    # the work a prefix-reusing forward needs: rows s0 .. K-1 of every x'
    # (s0 = K-1 for x' = x), each row s attending to s + 1 keys
    K = d["K"]
    xk = keys.cpu().numpy().view(np.uint64)
    xp = con["xprime"].cpu().numpy().view(np.uint64)
    d0, d1 = xk[:, None, 0] ^ xp[..., 0], xk[:, None, 1] ^ xp[..., 1]

    def bitlen(v):  # bit length of uint64 values, exactly (32-bit halves in float64)
        hi, lo = (v >> np.uint64(32)).astype(np.float64), (v & np.uint64(0xFFFFFFFF)).astype(np.float64)
        return np.where(hi > 0, 32 + np.frexp(hi)[1], np.frexp(lo)[1])

    top = np.where(d1 != 0, 64 + bitlen(d1) - 1, bitlen(d0) - 1)  # highest differing bit, -1 for x' = x
    s0 = np.where(top >= 0, K - 1 - (top // 2), K - 1).astype(np.int64)
    assert st["evaluated_rows"] == int(np.sum(K - s0))
    assert st["evaluated_keys"] == int(np.sum(K * (K + 1) // 2 - s0 * (s0 + 1) // 2))
    err = np.abs(g - ref) / absum
    print(f"prefix vs whole-forward {prec} K={d['K']}: max |dE|/A = {err.max():.3e}")
    assert err.max() <= 1e-12


def test_bf16_eloc_model_chunks_and_tail(nn):
    """More samples than one prefix-cache chunk at a small C (N=8, 27
    connections: 4,096 samples per chunk), ragged tail; equal to the
    whole-forward assembly as above."""
    d = synth.config_inputs(2, K=4, n_up=2, n_dn=2, n_unique=30, model=True)
    _print_case("bf16_chunks")
    S = nn.System(d["N"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"])
    M = nn.Model(d["model_shape"], d["n_up"], d["n_dn"], d["weights"])
    rng = np.random.default_rng(7)
    idx = rng.integers(0, len(d["keys"]), size=5000)   # repeated samples are fine for the full path
    k = d["keys"][idx]
    keys, cnt = dev(k), dev(np.ones(len(k), np.uint32), torch.int32)
    e, _, _ = nn.eloc_model(S, M, keys, cnt, nn.NNQS_BF16)
    ref, _, _ = nn.eloc_model(S, M, keys[:7].contiguous(), cnt[:7].contiguous(), nn.NNQS_BF16)
    torch.cuda.synchronize()
    g = eloc_complex(e)
    first = {}
    for i, kk in enumerate(idx):
        first.setdefault(int(kk), i)
    for i, kk in enumerate(idx):
        assert g[i] == g[first[int(kk)]], i
    assert np.allclose(g[:7], eloc_complex(ref), rtol=0, atol=0)


@pytest.mark.parametrize("kw", [dict(cfg=3, n_unique=16), dict(cfg=2, K=16, n_up=3, n_dn=5, n_unique=37, model=True)])
def test_logpsi_fp8_error_vs_oracle(nn, kw):
    """FP8 rung of the network: the four weight products on
    v_mfma_f32_16x16x32_fp8_fp8 (OCP E4M3, power-of-two weight scales), the
    attention and the phase MLP as in BF16.  The error against the FP64
    oracle is stated and bounded by 0.5 + 0.02 |log|psi|| nats."""
    kw = dict(kw)
    cfg = kw.pop("cfg")
    d = synth.config_inputs(cfg, **kw)
    _print_case("logpsi_fp8", K=d["K"])
    shape, w = d["model_shape"], d["weights"]
    M = nn.Model(shape, d["n_up"], d["n_dn"], w)
    keys = d["keys"] if d["K"] < 60 else np.concatenate([d["keys"], _random_connected(d, 2, 500, 9)])
    la8, _ = nn.model_logpsi(M, dev(keys), nn.NNQS_FP8)
    la16, _ = nn.model_logpsi(M, dev(keys), nn.NNQS_BF16)
    torch.cuda.synchronize()
    ola, _ = oracle.net_logpsi(w, shape, d["n_up"], d["n_dn"], keys)
    d8, d16 = np.abs(la8.cpu().numpy() - ola), np.abs(la16.cpu().numpy() - ola)
    print(f"FP8 vs FP64 oracle K={d['K']}: max |dlogabs| {d8.max():.3e} (mean {d8.mean():.3e}); "
          f"BF16 max {d16.max():.3e} (mean {d16.mean():.3e}); n={len(keys)}")
    assert np.all(d8 <= 0.5 + 0.02 * np.abs(ola))


@pytest.mark.parametrize("prec,case", [("bf16", "sampled"), ("fp8", "sampled"), ("bf16", "sector")])
def test_dedup_evaluates_each_distinct_xprime_once(nn, prec, case):
    """With dedup every distinct x' of the chunk goes through the forward
    once (from the sample whose first change is latest) and its amplitude is
    copied to every connection that reaches it: E_loc equals the per-
    connection evaluation up to FP64 summation order, and the forward's
    distinct count is the number of distinct keys among the connections.
    The whole-sector case takes every determinant as a sample, so each x'
    is reached from every sample it connects to (runs of up to C equal
    keys in the sorted list)."""
    if case == "sector":
        d = synth.config_inputs(1, K=7, n_up=3, n_dn=2, model=True)
    else:
        d = synth.config_inputs(2, K=16, n_up=4, n_dn=4, n_unique=40, model=True)
    P = nn.NNQS_BF16 if prec == "bf16" else nn.NNQS_FP8
    _print_case("dedup", K=d["K"], prec=prec, case=case, n=d["keys"].shape[0])
    S = nn.System(d["N"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"])
    M = nn.Model(d["model_shape"], d["n_up"], d["n_dn"], d["weights"])
    keys, cnt = dev(d["keys"]), dev(d["counts"], torch.int32)
    e0, en0, st0 = nn.eloc_model(S, M, keys, cnt, P, with_stats=True)
    e1, en1, st1 = nn.eloc_model(S, M, keys, cnt, P, with_stats=True, dedup=True)
    con = nn.connections(S, keys)
    torch.cuda.synchronize()
    xp = con["xprime"].cpu().numpy().reshape(-1, 2)
    distinct = np.unique(xp.view([("a", np.int64), ("b", np.int64)])).shape[0]
    print(f"dedup {prec}: {st1['evaluated']} connections, {st1['evaluated_distinct']} distinct "
          f"(rows {st0['evaluated_rows']} -> {st1['evaluated_rows']})")
    assert st1["evaluated"] == st0["evaluated"] == keys.shape[0] * S.connection_count
    assert st1["evaluated_distinct"] == distinct < st1["evaluated"]
    assert sum(st1["evaluated_class"]) == distinct
    assert st1["evaluated_rows"] < st0["evaluated_rows"]
    # scale of each E_loc: sum of |terms| from the whole-sequence amplitudes
    C = S.connection_count
    xla, _ = nn.model_logpsi(M, con["xprime"].reshape(-1, 2), P)
    sla, _ = nn.model_logpsi(M, keys, P)
    torch.cuda.synchronize()
    absum = (np.abs(con["hxx"].cpu().numpy())
             * np.exp(xla.cpu().numpy().reshape(-1, C) - sla.cpu().numpy()[:, None])).sum(axis=1)
    a, b = eloc_complex(e0), eloc_complex(e1)
    err = np.abs(a - b) / absum
    print(f"dedup vs per-connection {prec}: max |dE|/A = {err.max():.3e}")
    assert err.max() <= 1e-12


@pytest.mark.parametrize("cfg,kw", [(2, dict(K=40, n_up=3, n_dn=3, n_unique=6, model=True)),
                                    (3, dict(n_unique=2))])
def test_dedup_with_every_term_refined_equals_fp64(nn, cfg, kw):
    """Dedup and the FP64 refinement together: with every term refined the
    result is the FP64 path's (each distinct x' refined once, from its
    representative's FP64 cache, and copied)."""
    d = synth.config_inputs(cfg, **kw)
    _print_case("dedup_refine_all", K=d["K"])
    S = nn.System(d["N"], d["n_up"], d["n_dn"], d["h"], d["g"], d["e_core"])
    M = nn.Model(d["model_shape"], d["n_up"], d["n_dn"], d["weights"])
    keys, cnt = dev(d["keys"]), dev(d["counts"], torch.int32)
    e64, _, _ = nn.eloc_model(S, M, keys, cnt, nn.NNQS_FP64)
    e, _, st = nn.eloc_model(S, M, keys, cnt, nn.NNQS_BF16, refine_nats=60.0, with_stats=True, dedup=True)
    torch.cuda.synchronize()
    a, b = eloc_complex(e64), eloc_complex(e)
    assert 0 < st["refined"] <= st["evaluated_distinct"] <= st["evaluated"]
    assert np.max(np.abs(a - b)) <= 1e-12 * max(1.0, np.abs(a).max())
