"""Pins of the oracle's batch autoregressive sampling (Section 3.1) and of
its counter-based generator, independent of the oracle's own code paths:
published known-answer vectors of Philox4x32-10, the sample distribution
against |psi|^2 over a whole sector, and invariants of the samples."""
import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("ctr,key,want", [
    # Known-answer vectors distributed with the Random123 library (Salmon et
    # al., SC 2011) for philox4x32 with 10 rounds.
    ([0, 0, 0, 0], [0, 0], [0x6627e8d5, 0xe169c58d, 0xbc57ac4c, 0x9b00dbd8]),
    ([0xffffffff] * 4, [0xffffffff] * 2, [0x408f276d, 0x41c83b0e, 0xa20bc7c6, 0x6d5451fd]),
    ([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344], [0xa4093822, 0x299f31d0],
     [0xd16cfe09, 0x94fdcceb, 0x5001e420, 0x24126ea1]),
])
def test_philox_known_answers(ctr, key, want):
    assert [int(v) for v in oracle.philox4x32_10(ctr, key)] == want


def test_bas_uniforms_are_uniform():
    u = np.array([oracle.bas_uniform(123, 5, i) for i in range(100000)])
    assert u.min() >= 0.0 and u.max() < 1.0
    assert abs(u.mean() - 0.5) < 0.004
    hist = np.histogram(u, bins=20, range=(0, 1))[0]
    assert np.all(np.abs(hist - 5000) < 5 * np.sqrt(5000))


def test_bas_samples_follow_psi_squared_over_a_sector():
    """K=4 (2 up, 2 down, 36 determinants): with 400,000 samples the
    frequencies match |psi|^2 from the network (normalised over the sector by
    the mask, Eq. 12) within five standard deviations."""
    d = synth.config_inputs(1, model=True)
    w, shape = d["weights"], d["model_shape"]
    keys, counts, la = oracle.bas(w, shape, d["n_up"], d["n_dn"], 400000, seed=11, capacity=64)
    assert counts.sum() == 400000
    allk = d["keys"]
    p_la, _ = oracle.net_logpsi(w, shape, d["n_up"], d["n_dn"], allk)
    p = np.exp(2.0 * p_la)
    assert abs(p.sum() - 1.0) < 1e-12
    freq = np.zeros(len(allk))
    index = {(int(a), int(b)): i for i, (a, b) in enumerate(allk)}
    for (a, b), c in zip(keys, counts):
        freq[index[(int(a), int(b))]] += c
    sigma = np.sqrt(400000 * p * (1 - p))
    assert np.all(np.abs(freq - 400000 * p) <= 5 * sigma + 1)


@pytest.mark.parametrize("kw", [dict(K=6, n_up=2, n_dn=3), dict(K=12, n_up=4, n_dn=3)])
def test_bas_invariants(kw):
    d = synth.config_inputs(2, n_unique=4, model=True, **kw)
    w, shape = d["weights"], d["model_shape"]
    keys, counts, la = oracle.bas(w, shape, d["n_up"], d["n_dn"], 50000, seed=3, capacity=1 << 16)
    assert counts.sum() == 50000 and counts.min() >= 1
    occ = synth.unpack_keys(keys, d["K"])
    assert np.all(occ[:, 0].sum(axis=1) == d["n_up"]) and np.all(occ[:, 1].sum(axis=1) == d["n_dn"])
    assert len({(int(a), int(b)) for a, b in keys}) == len(keys)
    ola, _ = oracle.net_logpsi(w, shape, d["n_up"], d["n_dn"], keys)
    assert np.max(np.abs(ola - la)) <= 1e-12 * np.max(np.abs(ola))
    k2, c2, _ = oracle.bas(w, shape, d["n_up"], d["n_dn"], 50000, seed=3, capacity=1 << 16)
    assert (k2 == keys).all() and (c2 == counts).all()
    k3, c3, _ = oracle.bas(w, shape, d["n_up"], d["n_dn"], 50000, seed=4, capacity=1 << 16)
    assert len(k3) != len(keys) or not (c3 == counts).all()
