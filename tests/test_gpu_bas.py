"""GPU batch autoregressive sampling (Section 3.1) against the FP64 oracle's:
with the FP64 network the unique samples, their order and counts are
bit-identical for the same seed (both sides draw from Philox4x32-10 at the
same counters); in BF16 the samples conserve the electron numbers, the
counts sum to the sample number and the path log-amplitudes equal the
network's own, and over a whole sector the frequencies follow |psi|^2."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests.gpu_util import keys_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nn():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_16705_amd as nn
    return nn


@pytest.mark.parametrize("kw,ns,seed", [(dict(cfg=1), 100000, 7), (dict(cfg=2, K=6, n_up=2, n_dn=3), 30001, 1),
                                        (dict(cfg=2, K=12, n_up=4, n_dn=3), 200000, 5),
                                        (dict(cfg=2, K=40, n_up=3, n_dn=2), 20000, 9)])
def test_bas_fp64_equals_oracle(nn, kw, ns, seed):
    kw = dict(kw)
    cfg = kw.pop("cfg")
    d = synth.config_inputs(cfg, model=True, **({} if cfg == 1 else dict(n_unique=4, **kw)))
    print(f"[case] bas_fp64 K={d['K']} n_samples={ns} seed={seed}", flush=True)
    M = nn.Model(d["model_shape"], d["n_up"], d["n_dn"], d["weights"])
    k, c, la, ph = nn.bas(M, ns, seed, nn.NNQS_FP64, capacity=1 << 17)
    torch.cuda.synchronize()
    ok, oc, ola = oracle.bas(d["weights"], d["model_shape"], d["n_up"], d["n_dn"], ns, seed, capacity=1 << 17)
    gk = keys_np(k)
    print(f"BAS K={d['K']}: {len(ok)} unique samples")
    assert gk.shape == ok.shape and (gk == ok).all()
    assert (c.cpu().numpy().astype(np.uint32) == oc).all()
    assert np.max(np.abs(la.cpu().numpy() - ola)) <= 1e-12 * max(1.0, np.abs(ola).max())
    _, oph = oracle.net_logpsi(d["weights"], d["model_shape"], d["n_up"], d["n_dn"], ok)
    assert np.max(np.abs(ph.cpu().numpy() - oph)) <= 1e-12


def test_bas_bf16_n120_invariants(nn):
    """N=120 (20 up + 20 down): 10^5 samples in BF16."""
    d = synth.config_inputs(3, n_unique=2)
    print("[case] bas_bf16 N=120", flush=True)
    M = nn.Model(d["model_shape"], d["n_up"], d["n_dn"], d["weights"])
    k, c, la, ph = nn.bas(M, 100000, 3, nn.NNQS_BF16)
    torch.cuda.synchronize()
    keys = keys_np(k)
    cnt = c.cpu().numpy().astype(np.int64)
    assert cnt.sum() == 100000 and cnt.min() >= 1
    occ = synth.unpack_keys(keys, d["K"])
    assert np.all(occ[:, 0].sum(axis=1) == 20) and np.all(occ[:, 1].sum(axis=1) == 20)
    assert len({(int(a), int(b)) for a, b in keys}) == len(keys)
    la2, _ = nn.model_logpsi(M, k.contiguous(), nn.NNQS_BF16)
    diff = np.abs(la.cpu().numpy() - la2.cpu().numpy())
    print(f"BAS BF16 N=120: {len(keys)} unique of 100000, path vs network log|psi| max diff {diff.max():.2e}")
    assert diff.max() <= 1e-5


def test_bas_bf16_frequencies_follow_psi_squared(nn):
    d = synth.config_inputs(1, model=True)
    M = nn.Model(d["model_shape"], d["n_up"], d["n_dn"], d["weights"])
    print("[case] bas_bf16 K=4 distribution", flush=True)
    k, c, la, _ = nn.bas(M, 1000000, 17, nn.NNQS_BF16, capacity=64)
    keys, cnt = keys_np(k), c.cpu().numpy().astype(np.float64)
    p = np.exp(2.0 * la.cpu().numpy())
    assert abs(p.sum() - 1.0) < 1e-3 and len(keys) == 36
    sigma = np.sqrt(1e6 * p * (1 - p))
    assert np.all(np.abs(cnt - 1e6 * p) <= 5 * sigma + 1)


def test_bas_errors(nn):
    d = synth.config_inputs(2, K=12, n_up=4, n_dn=3, n_unique=4, model=True)
    M = nn.Model(d["model_shape"], d["n_up"], d["n_dn"], d["weights"])
    with pytest.raises(nn.NNQSError) as ei:
        nn.bas(M, 100000, 1, nn.NNQS_FP64, capacity=8)
    assert ei.value.code == -4
    with pytest.raises(nn.NNQSError):
        nn.bas(M, 0, 1, nn.NNQS_FP64)
