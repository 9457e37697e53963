"""Pins of the VMC-gradient oracle (oracle/vmc.py).

* its float64 forward equals the C oracle's network forward (an independent
  implementation, itself pinned in test_oracle_net_pins.py) to 1e-12;
* its parameter gradients equal central finite differences of the C oracle's
  forward, tensor by tensor (a dropped term, a wrong sign or a transposed
  operand in any tensor's gradient fails its own check);
* Eq. 7 with the exact distribution p = |psi|^2 over a whole sector equals
  the finite-difference gradient of the exact energy <psi|H|psi>/<psi|psi>,
  with H the dense Jordan-Wigner matrix (tests/jw_bruteforce.py): this pins
  the factor 2, the subtracted mean and the sign of the phase term;
* Eq. 13: linear warm-up, peak at the warm-up length, i^-1/2 decay after it;
* AdamW equals torch.optim.AdamW (the library routine) over several steps.
"""
import numpy as np
import pytest
import torch

import oracle
import oracle.vmc as vmc
import synth
from tests import jw_bruteforce as jw


def _small(K, nu, nd, seed=11, L=2, d=16, F=32, P=24, std=0.2):
    shape = synth.TransformerShape(K=K, d_model=d, n_layers=L, n_heads=4, d_ff=F, phase_hidden=P)
    rng = np.random.default_rng([synth.SEED_ROOT, 902, seed])
    w = synth.transformer_weights(shape, nu, nd, rng, beta=0.6, std=std)
    return shape, {k: np.asarray(v, dtype=np.float64) for k, v in w.items()}


@pytest.mark.parametrize("K,nu,nd,L,d,F,P", [(5, 2, 2, 2, 16, 32, 24), (8, 3, 3, 4, 64, 256, 512),
                                              (60, 20, 20, 4, 64, 256, 512)])
def test_forward_matches_c_oracle(K, nu, nd, L, d, F, P):
    shape, w = _small(K, nu, nd, L=L, d=d, F=F, P=P, std=0.02 if d == 64 else 0.2)
    if K <= 8:
        keys = synth.all_determinants(K, nu, nd)[:64]
    else:
        keys, _ = synth.geometric_samples(K, nu, nd, 4, np.random.default_rng(5))
    la, ph = vmc.logpsi(w, shape, nu, nd, keys)
    cla, cph = oracle.net_logpsi(w, shape, nu, nd, keys)
    assert np.max(np.abs(la - cla)) < 1e-12 * max(1.0, np.abs(cla).max())
    assert np.max(np.abs(ph - cph)) < 1e-12


def _c_objective(w, shape, nu, nd, keys, cl, cp):
    la, ph = oracle.net_logpsi(w, shape, nu, nd, keys)
    return float(cl @ la + cp @ ph)


def test_vjp_matches_finite_differences_per_tensor():
    K, nu, nd = 5, 2, 2
    shape, w = _small(K, nu, nd)
    keys = synth.all_determinants(K, nu, nd)[::3]
    rng = np.random.default_rng(4)
    cl = rng.normal(size=len(keys))
    cp = rng.normal(size=len(keys))
    g = vmc.logpsi_vjp(w, shape, nu, nd, keys, cl, cp)
    assert np.all(g["logit_bias"] == 0.0)
    h = 1e-5
    for name in oracle.net_order(shape.n_layers):
        if name in vmc.FIXED:
            continue
        u = rng.normal(size=w[name].shape)
        u /= np.linalg.norm(u)
        wp = dict(w)
        wm = dict(w)
        wp[name] = w[name] + h * u
        wm[name] = w[name] - h * u
        fd = (_c_objective(wp, shape, nu, nd, keys, cl, cp) - _c_objective(wm, shape, nu, nd, keys, cl, cp)) / (2 * h)
        an = float(np.sum(g[name] * u))
        assert abs(fd - an) < 1e-7 * max(1.0, abs(fd)), (name, fd, an)


def test_vjp_single_entries():
    """Entry-wise derivative of one configuration's log|psi| and phase."""
    K, nu, nd = 6, 2, 3
    shape, w = _small(K, nu, nd, seed=12)
    keys = synth.all_determinants(K, nu, nd)[5:6]
    for which, (cl, cp) in (("logabs", ([1.0], [0.0])), ("phase", ([0.0], [1.0]))):
        g = vmc.logpsi_vjp(w, shape, nu, nd, keys, cl, cp)
        rng = np.random.default_rng(9)
        for name in ("tok_emb", "pos_emb", "l0.wq", "l1.bv", "l1.w2", "lnf_g", "head_w", "head_b",
                     "ph_w1", "ph_b2", "ph_w3", "ph_b3"):
            idx = tuple(int(rng.integers(s)) for s in w[name].shape)
            h = 1e-6
            wp, wm = dict(w), dict(w)
            wp[name] = w[name].copy()
            wm[name] = w[name].copy()
            wp[name][idx] += h
            wm[name][idx] -= h
            fd = (_c_objective(wp, shape, nu, nd, keys, np.array(cl), np.array(cp)) -
                  _c_objective(wm, shape, nu, nd, keys, np.array(cl), np.array(cp))) / (2 * h)
            assert abs(fd - g[name][idx]) < 1e-7 * max(1.0, abs(fd)), (which, name, idx, fd, g[name][idx])


def _exact_energy(w, shape, nu, nd, Hs, keys):
    la, ph = oracle.net_logpsi(w, shape, nu, nd, keys)
    psi = np.exp(la + 1j * ph)
    return float(np.real(np.vdot(psi, Hs @ psi) / np.vdot(psi, psi)))


def test_eq7_is_the_gradient_of_the_exact_energy():
    K, nu, nd = 4, 2, 1
    rng = np.random.default_rng([synth.SEED_ROOT, 903])
    h1, g2, _ = synth.integrals(K, rng)
    Hs, idx = jw.sector_hamiltonian(K, nu, nd, h1, g2, 0.7)
    Hs = np.asarray(Hs.todense() if hasattr(Hs, "todense") else Hs)
    keys = np.stack([jw.index_to_key(int(b)) for b in idx])
    shape, w = _small(K, nu, nd, seed=13, std=0.3)
    la, ph = oracle.net_logpsi(w, shape, nu, nd, keys)
    psi = np.exp(la + 1j * ph)
    p = np.abs(psi) ** 2
    assert abs(p.sum() - 1.0) < 1e-12                       # autoregressive normalisation
    eloc = (Hs @ psi) / psi                                 # Eq. 4 by the dense matrix
    g, E = vmc.vmc_gradient(w, shape, nu, nd, keys, p, eloc)
    assert abs(E.imag) < 1e-12
    assert abs(E.real - _exact_energy(w, shape, nu, nd, Hs, keys)) < 1e-12
    h = 1e-5
    for name in oracle.net_order(shape.n_layers):
        if name in vmc.FIXED:
            continue
        u = rng.normal(size=w[name].shape)
        u /= np.linalg.norm(u)
        wp, wm = dict(w), dict(w)
        wp[name] = w[name] + h * u
        wm[name] = w[name] - h * u
        fd = (_exact_energy(wp, shape, nu, nd, Hs, keys) - _exact_energy(wm, shape, nu, nd, Hs, keys)) / (2 * h)
        an = float(np.sum(g[name] * u))
        assert abs(fd - an) < 1e-7 * max(1.0, abs(fd)), (name, fd, an)


def test_eq7_mean_subtraction_and_weights():
    """Adding a constant to every local energy leaves Eq. 7 unchanged; equal
    counts behave as equal probabilities."""
    K, nu, nd = 5, 2, 2
    shape, w = _small(K, nu, nd, seed=14)
    keys = synth.all_determinants(K, nu, nd)[:12]
    rng = np.random.default_rng(2)
    eloc = rng.normal(size=12) + 1j * rng.normal(size=12)
    counts = rng.integers(1, 9, size=12)
    g1, E1 = vmc.vmc_gradient(w, shape, nu, nd, keys, counts, eloc)
    g2, E2 = vmc.vmc_gradient(w, shape, nu, nd, keys, 3 * counts, eloc + (5.0 - 2.0j))
    assert abs(E2 - E1 - (5.0 - 2.0j)) < 1e-12
    for k in g1:
        assert np.allclose(g1[k], g2[k], rtol=1e-11, atol=1e-14)


def test_lr_schedule_eq13():
    d, S = 64, 4000
    lr = [vmc.lr_schedule(i, d, S) for i in range(1, 20001)]
    peak = int(np.argmax(lr)) + 1
    assert peak == S
    assert abs(lr[S - 1] - 1.0 / (8.0 * np.sqrt(S))) < 1e-18   # d^-1/2 = 1/8
    assert abs(lr[0] * 1000 - lr[999]) < 1e-18                  # linear warm-up
    assert abs(vmc.lr_schedule(4 * 5000, d, S) * 2 - vmc.lr_schedule(5000, d, S)) < 1e-18  # i^-1/2 decay


def test_adamw_matches_torch():
    rng = np.random.default_rng(3)
    n = 257
    w = rng.normal(size=n)
    m = np.zeros(n)
    v = np.zeros(n)
    p = torch.tensor(w.copy(), requires_grad=True)
    opt = torch.optim.AdamW([p], lr=2e-3, betas=(0.9, 0.98), eps=1e-9, weight_decay=0.05)
    for t in range(1, 6):
        g = rng.normal(size=n)
        w, m, v = vmc.adamw_step(w, g, m, v, t, 2e-3, 0.9, 0.98, 1e-9, 0.05)
        p.grad = torch.tensor(g)
        opt.step()
        assert np.max(np.abs(w - p.detach().numpy())) < 1e-14


def test_adamw_leaves_fixed_entries():
    w = np.arange(6, dtype=np.float64)
    g = np.ones(6)
    mask = np.array([1, 1, 0, 1, 0, 1], dtype=np.float64)
    nw, m, v = vmc.adamw_step(w, g, np.zeros(6), np.zeros(6), 1, 0.1, 0.9, 0.999, 1e-8, 0.01, mask)
    assert nw[2] == w[2] and nw[4] == w[4]
    assert np.all(nw[mask == 1] < w[mask == 1])
