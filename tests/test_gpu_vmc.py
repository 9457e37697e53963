"""GPU VMC gradient step against the FP64 oracle (oracle/vmc.py):

* the weighted parameter gradient (every tensor of the layout) at K = 4, 8
  (several 256-configuration passes) and at the N=120 shape (K = 60);
* the Eq. 7 gradient and its energy;
* AdamW with the Eq. 13 learning rate, the FP64 forward after the update and
  the rebuilt BF16 copy;
* one whole VMC iteration (sampling, local energies, gradient, update) in
  FP64 against the same chain in the oracle.
The backward is FP64 with its own summation order: the bar is 1e-10 of the
largest gradient entry of each tensor (1e-9 at K = 60)."""
import numpy as np
import pytest
import torch

import oracle
import oracle.vmc as vmc
import synth
from tests.gpu_util import dev, keys_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def nn():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2306_16705_amd as nn
    return nn


def _inputs(K, nu, nd, n, seed=0):
    if K <= 8:
        d = synth.config_inputs(2, K=K, n_up=nu, n_dn=nd, n_unique=4, model=True)
        keys = synth.all_determinants(K, nu, nd)[:n]
    else:
        d = synth.config_inputs(3, n_unique=n)
        keys = d["keys"][:n]
    return d, np.ascontiguousarray(keys)


def _compare(flat_gpu, ora: dict, shape, rel, label):
    """Per tensor: |gpu - oracle| <= rel * (largest entry of the tensor) +
    1e-13 * (largest entry of the whole gradient).  The second term covers
    tensors whose gradient vanishes identically, such as the key bias (a
    shift of every score of a query leaves its softmax unchanged): both sides
    then return rounding noise."""
    g = vmc.unpack(flat_gpu, ora, shape)
    gscale = max(float(np.abs(v).max()) for v in ora.values())
    worst = 0.0
    for k in oracle.net_order(shape.n_layers):
        scale = max(1e-300, float(np.abs(ora[k]).max()))
        err = float(np.abs(g[k] - ora[k]).max())
        if k in vmc.FIXED:
            assert err == 0.0 and np.all(g[k] == 0.0), k
            continue
        assert err <= rel * scale + 1e-13 * gscale, f"{label}: {k} err {err:.3e} scale {scale:.3e}"
        if scale > 1e-10 * gscale:
            worst = max(worst, err / scale)
    return worst


@pytest.mark.parametrize("K,nu,nd,n", [(4, 2, 2, 36), (8, 3, 3, 600), (60, 20, 20, 6)])
def test_model_grad_matches_oracle(nn, K, nu, nd, n):
    d, keys = _inputs(K, nu, nd, n)
    shape = d["model_shape"]
    n = len(keys)
    print(f"[case] model_grad K={K} n={n}", flush=True)
    rng = np.random.default_rng([K, n])
    cl = rng.normal(size=n)
    cp = rng.normal(size=n)
    M = nn.Model(shape, d["n_up"], d["n_dn"], d["weights"])
    g, la, ph = nn.model_grad(M, dev(keys), dev(cl), dev(cp), with_values=True)
    g2 = nn.model_grad(M, dev(keys), dev(cl), dev(cp))
    torch.cuda.synchronize()
    assert torch.equal(g, g2), "two calls differ"
    ola, oph = oracle.net_logpsi(d["weights"], shape, d["n_up"], d["n_dn"], keys)
    assert np.max(np.abs(la.cpu().numpy() - ola)) <= 1e-12 * max(1.0, np.abs(ola).max())
    assert np.max(np.abs(ph.cpu().numpy() - oph)) <= 1e-12
    ora = vmc.logpsi_vjp(d["weights"], shape, d["n_up"], d["n_dn"], keys, cl, cp)
    worst = _compare(g.cpu().numpy(), ora, shape, 1e-9 if K > 8 else 1e-10, f"K={K}")
    print(f"model grad K={K} n={n}: max error / tensor scale {worst:.2e}")


def test_vmc_gradient_matches_oracle(nn):
    K, nu, nd = 6, 2, 3
    d, keys = _inputs(K, nu, nd, 100)
    shape = d["model_shape"]
    n = len(keys)
    print(f"[case] vmc_gradient K={K} n={n}", flush=True)
    rng = np.random.default_rng(8)
    counts = rng.integers(1, 40, size=n).astype(np.uint32)
    eloc = rng.normal(-5.0, 1.0, size=n) + 1j * rng.normal(0.0, 0.1, size=n)
    e2 = np.stack([eloc.real, eloc.imag], axis=1)
    M = nn.Model(shape, d["n_up"], d["n_dn"], d["weights"])
    g, en = nn.vmc_gradient(M, dev(keys), dev(counts.view(np.int32)), dev(e2))
    torch.cuda.synchronize()
    ora, E = vmc.vmc_gradient(d["weights"], shape, d["n_up"], d["n_dn"], keys, counts, eloc)
    en = en.cpu().numpy()
    assert abs(en[0] - E.real) < 1e-12 * abs(E.real) and abs(en[1] - E.imag) < 1e-12
    assert en[2] == counts.sum()
    worst = _compare(g.cpu().numpy(), ora, shape, 1e-10, "vmc")
    print(f"VMC gradient K={K}: max error / tensor scale {worst:.2e}")


def test_adamw_matches_oracle_and_refreshes_copies(nn):
    K, nu, nd = 6, 2, 3
    d, keys = _inputs(K, nu, nd, 60)
    shape = d["model_shape"]
    n = len(keys)
    print(f"[case] adamw K={K}", flush=True)
    M = nn.Model(shape, d["n_up"], d["n_dn"], d["weights"])
    w = oracle.pack_net(d["weights"], shape)
    mask = vmc.fixed_mask(d["weights"], shape)
    nw = w.size
    m1 = torch.zeros(nw, dtype=torch.float64, device="cuda")
    m2 = torch.zeros(nw, dtype=torch.float64, device="cuda")
    om1, om2 = np.zeros(nw), np.zeros(nw)
    rng = np.random.default_rng(5)
    for t in range(1, 4):
        g = rng.normal(size=nw) * 1e-2
        lr = nn.lr_schedule(t, shape.d_model, 4000)
        assert lr == pytest.approx(vmc.lr_schedule(t, shape.d_model, 4000), rel=1e-15)
        lr *= 100.0  # a visible step at this tiny iteration count
        nn.model_adamw_step(M, dev(g), t, lr, m1, m2, 0.9, 0.98, 1e-9, 0.05)
        w, om1, om2 = vmc.adamw_step(w, g, om1, om2, t, lr, 0.9, 0.98, 1e-9, 0.05, mask)
    gw = nn.model_get_weights(M).cpu().numpy()
    torch.cuda.synchronize()
    assert np.max(np.abs(gw - w)) <= 1e-15 * max(1.0, np.abs(w).max())
    assert np.max(np.abs(m1.cpu().numpy() - om1)) <= 1e-16 and np.max(np.abs(m2.cpu().numpy() - om2)) <= 1e-18
    wd = vmc.unpack(w, d["weights"], shape)
    ola, oph = oracle.net_logpsi(wd, shape, d["n_up"], d["n_dn"], keys)
    la, ph = nn.model_logpsi(M, dev(keys), nn.NNQS_FP64)
    assert np.max(np.abs(la.cpu().numpy() - ola)) <= 1e-12 * max(1.0, np.abs(ola).max())
    assert np.max(np.abs(ph.cpu().numpy() - oph)) <= 1e-12
    lb, pb = nn.model_logpsi(M, dev(keys), nn.NNQS_BF16)
    err = np.max(np.abs(lb.cpu().numpy() - ola))
    print(f"AdamW: BF16 copy after 3 steps max |dlogabs| {err:.2e} vs the updated FP64 network (n={n})")
    assert err <= 2e-2


def test_one_vmc_iteration_fp64_equals_oracle(nn):
    """Sampling (FP64 BAS), full local energies (FP64), Eq. 7, AdamW with the
    Eq. 13 rate: the GPU chain against the oracle's, then the energy of the
    updated network."""
    K, nu, nd = 6, 2, 3
    d = synth.config_inputs(2, K=K, n_up=nu, n_dn=nd, n_unique=4, model=True)
    shape, W = d["model_shape"], d["weights"]
    print("[case] vmc_iteration K=6", flush=True)
    M = nn.Model(shape, nu, nd, W)
    S = nn.System(d["N"], nu, nd, d["h"], d["g"], d["e_core"])
    k, c, _, _ = nn.bas(M, 5000, 21, nn.NNQS_FP64, capacity=4096)
    e, en, _ = nn.eloc_model(S, M, k.contiguous(), c.contiguous(), nn.NNQS_FP64)
    g, en2 = nn.vmc_gradient(M, k.contiguous(), c.contiguous(), e)
    nw = g.numel()
    m1 = torch.zeros(nw, dtype=torch.float64, device="cuda")
    m2 = torch.zeros(nw, dtype=torch.float64, device="cuda")
    lr = nn.lr_schedule(1, shape.d_model, 4000) * 1000.0
    # eps 1e-3: Adam divides by |g| + eps, which would magnify the 1e-12
    # differences of the two local-energy paths for entries with |g| ~ eps
    nn.model_adamw_step(M, g, 1, lr, m1, m2, 0.9, 0.999, 1e-3, 0.01)
    gw = nn.model_get_weights(M).cpu().numpy()
    torch.cuda.synchronize()
    ok, oc, _ = oracle.bas(W, shape, nu, nd, 5000, 21, capacity=4096)
    assert (keys_np(k) == ok).all() and (c.cpu().numpy().astype(np.uint32) == oc).all()
    oe = oracle.eloc_model(K, nu, nd, d["h"], d["g"], d["e_core"], W, shape, ok)
    og, E = vmc.vmc_gradient(W, shape, nu, nd, ok, oc, oe)
    assert abs(en2.cpu().numpy()[0] - E.real) <= 1e-11 * abs(E.real)
    w0 = oracle.pack_net(W, shape)
    ow, _, _ = vmc.adamw_step(w0, vmc.pack(og, shape), np.zeros(nw), np.zeros(nw), 1, lr, 0.9, 0.999, 1e-3, 0.01,
                              vmc.fixed_mask(W, shape))
    assert np.max(np.abs(gw - ow)) <= 1e-8 * lr
    # the exact energy of the sector before and after the step (reported)
    keys = synth.all_determinants(K, nu, nd)
    def exact_energy(wflat):
        wd = vmc.unpack(wflat, W, shape)
        la, ph = oracle.net_logpsi(wd, shape, nu, nd, keys)
        el = oracle.eloc_model(K, nu, nd, d["h"], d["g"], d["e_core"], wd, shape, keys)
        return float(np.sum(np.exp(2 * la) * el.real))
    e0, e1 = exact_energy(w0), exact_energy(ow)
    print(f"one VMC iteration K=6: {len(ok)} unique samples, E(sampled) {E.real:.6f}, "
          f"exact {e0:.6f} -> {e1:.6f}")


def test_grad_errors(nn):
    d = synth.config_inputs(2, K=6, n_up=2, n_dn=3, n_unique=4, model=True)
    M = nn.Model(d["model_shape"], 2, 3, d["weights"])
    keys = dev(synth.all_determinants(6, 2, 3)[:4])
    z = torch.zeros(4, dtype=torch.float64, device="cuda")
    nw = oracle.pack_net(d["weights"], d["model_shape"]).size
    zw = [torch.zeros(nw, dtype=torch.float64, device="cuda") for _ in range(3)]
    print("[case] vmc error paths", flush=True)
    with pytest.raises(nn.NNQSError):
        nn.model_adamw_step(M, zw[0], 0, 1e-3, zw[1], zw[2])          # step counts from 1
    with pytest.raises(nn.NNQSError):
        nn.model_adamw_step(M, zw[0], 1, 1e-3, zw[1], zw[2], beta1=1.0)
    assert nn.lr_schedule(0, 64, 4000) == 0.0
    g = nn.model_grad(M, keys, z, z)  # zero cotangents give a zero gradient
    torch.cuda.synchronize()
    assert float(g.abs().max()) == 0.0
