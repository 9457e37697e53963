"""Pins of the FP64 oracle against what the paper and the mathematics fix.

* a hand-derived two-electron Hamiltonian (golden fixture, Eq. 9);
* the literal Jordan-Wigner brute force of Eq. 9 (dense sector matrices);
* the definition of Eq. 4 evaluated by a dense matrix-vector product;
* the full-space identity of Eq. 3 -> Eq. 5 (energy = sum |psi|^2 E_loc / sum |psi|^2);
* the zero-variance property of an eigenvector;
* the closed-form connection count and the textbook Hartree-Fock energy;
* Hermiticity and particle/spin conservation;
* library routines (lexsort, searchsorted) for the sorted table.
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle
import synth
from tests import jw_bruteforce as jw

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _expand_g(K, uniq):
    g = np.zeros((K, K, K, K))
    for key, v in uniq.items():
        p, q, r, s = (int(c) for c in key)
        for (a, b, c, d) in {(p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                             (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)}:
            g[a, b, c, d] = v
    return g


def _key_of_index(b):
    b = int(b)
    return np.array([b & 0xFFFFFFFFFFFFFFFF, b >> 64], dtype=np.uint64)


def _index_of_key(k):
    return int(k[0]) | (int(k[1]) << 64)


def _closed_form_C(K, nu, nd):
    vu, vd = K - nu, K - nd
    return (1 + nu * vu + nd * vd + math.comb(nu, 2) * math.comb(vu, 2)
            + math.comb(nd, 2) * math.comb(vd, 2) + nu * vu * nd * vd)


def _small_system(K, nu, nd, seed, decay=None):
    rng = np.random.default_rng([synth.SEED_ROOT, 900, seed])
    h, g, ec = synth.integrals(K, rng, decay=decay)
    return h, g, 0.37 if seed % 2 else ec  # a nonzero core energy on odd seeds


# ----------------------------------------------------------------- golden
def test_golden_two_electron_matrix():
    d = json.load(open(os.path.join(GOLDEN, "k2_one_up_one_down.json")))
    K = d["K"]
    h = np.array(d["h"])
    g = _expand_g(K, d["g_unique"])
    H = np.array(d["H"])
    keys = d["basis_keys"]
    for a, ka in enumerate(keys):
        for b, kb in enumerate(keys):
            v, _ = oracle.hxx(K, h, g, d["e_core"], _key_of_index(kb), _key_of_index(ka))
            assert v == H[a, b], (ka, kb, v, H[a, b])
    # the brute force reproduces the same hand-derived matrix
    Hs, idx = jw.sector_hamiltonian(K, d["n_up"], d["n_dn"], h, g, d["e_core"])
    assert list(idx) == keys
    np.testing.assert_allclose(Hs.real, H, atol=1e-15)
    assert np.abs(Hs.imag).max() == 0.0


# ----------------------------------------------- Slater-Condon vs brute force
@pytest.mark.parametrize("K,nu,nd,seed", [(4, 2, 2, 1), (4, 2, 2, 2), (5, 2, 1, 3), (5, 3, 2, 4), (4, 1, 3, 5)])
def test_matrix_elements_match_jordan_wigner(K, nu, nd, seed):
    h, g, ec = _small_system(K, nu, nd, seed)
    Hs, idx = jw.sector_hamiltonian(K, nu, nd, h, g, ec)
    assert np.abs(Hs.imag).max() < 1e-14
    Hs = Hs.real
    scale = np.abs(Hs).max()
    for a, ba in enumerate(idx):          # row: bra x'
        for b, bb in enumerate(idx):      # column: ket x
            v, s = oracle.hxx(K, h, g, ec, _key_of_index(bb), _key_of_index(ba))
            assert abs(v - Hs[a, b]) <= 1e-12 * scale, (ba, bb, v, Hs[a, b])


@pytest.mark.parametrize("K,nu,nd,seed", [(4, 2, 2, 1), (5, 2, 1, 3), (5, 3, 2, 4)])
def test_enumeration_is_complete(K, nu, nd, seed):
    """Canonical enumeration = every sector configuration within two
    excitations, each exactly once; its H column equals the brute force."""
    h, g, ec = _small_system(K, nu, nd, seed)
    Hs, idx = jw.sector_hamiltonian(K, nu, nd, h, g, ec)
    pos = {int(b): i for i, b in enumerate(idx)}
    C = _closed_form_C(K, nu, nd)
    assert oracle.n_connections(K, nu, nd) == C
    for b in idx:
        x = _key_of_index(int(b))
        xp, sign, exc, hv = oracle.connections(K, nu, nd, h, g, ec, x)
        assert xp.shape[0] == C
        got = [_index_of_key(k) for k in xp]
        assert len(set(got)) == C
        expect = {int(y) for y in idx if bin(int(y) ^ int(b)).count("1") <= 4}
        assert set(got) == expect
        assert got[0] == int(b) and tuple(exc[0]) == (255, 255, 255, 255)
        col = Hs[:, pos[int(b)]].real
        for k, y in enumerate(got):
            assert abs(hv[k] - col[pos[y]]) <= 1e-12 * np.abs(Hs).max()
        # the rest of the column vanishes
        mask = np.ones(len(idx), bool)
        mask[[pos[y] for y in got]] = False
        assert np.abs(col[mask]).max(initial=0.0) < 1e-14


def test_canonical_order_and_exc_indices():
    K, nu, nd = 5, 2, 2
    h, g, ec = _small_system(K, nu, nd, 7)
    x = synth.hf_key(K, nu, nd)
    xp, sign, exc, hv = oracle.connections(K, nu, nd, h, g, ec, x)
    occ = {0: [0, 2], 1: [1, 3]}
    vir = {0: [4, 6, 8], 1: [5, 7, 9]}
    expect = [(255, 255, 255, 255)]
    for s in (0, 1):
        for q in occ[s]:
            for p in vir[s]:
                expect.append((q, 255, p, 255))
    for s in (0, 1):
        for i, j in itertools.combinations(occ[s], 2):
            for a, b in itertools.combinations(vir[s], 2):
                expect.append((i, j, a, b))
    for i in occ[0]:
        for a in vir[0]:
            for j in occ[1]:
                for b in vir[1]:
                    expect.append((min(i, j), max(i, j), min(a, b), max(a, b)))
    assert [tuple(e) for e in exc] == expect
    for k, e in enumerate(expect):
        y = x.copy()
        for p in e:
            if p != 255:
                y[p >> 6] ^= np.uint64(1) << np.uint64(p & 63)
        assert (xp[k] == y).all()


# --------------------------------------------------------- local energy pins
def _eloc_brute(Hs, psi):
    """Eq. 4 by definition: E_loc(x) = (H psi)(x) / psi(x), H[x, x'] = <x|H|x'>."""
    return (Hs @ psi) / psi


@pytest.mark.parametrize("cfg_kw", [dict(), dict(K=5, n_up=2, n_dn=1)])
def test_eloc_definition_and_fci_identity(cfg_kw):
    d = synth.config_inputs(1, **cfg_kw)
    K, nu, nd = d["K"], d["n_up"], d["n_dn"]
    Hs, idx = jw.sector_hamiltonian(K, nu, nd, d["h"], d["g"], d["e_core"])
    Hs = Hs.real
    pos = {int(b): i for i, b in enumerate(idx)}
    order = np.array([pos[_index_of_key(k)] for k in d["keys"]])
    psi = np.exp(d["logabs"] + 1j * d["phase"])
    psi_sector = np.zeros(len(idx), complex)
    psi_sector[order] = psi
    e = oracle.eloc_table(K, nu, nd, d["h"], d["g"], d["e_core"], d["keys"], d["logabs"], d["phase"],
                          d["keys"], d["logabs"], d["phase"])
    ref = _eloc_brute(Hs, psi_sector)[order]
    scale = np.maximum(1.0, np.abs(ref))
    assert np.all(np.abs(e - ref) <= 1e-12 * scale * np.abs(Hs).max())
    # Eq. 3 -> Eq. 5: <psi|H|psi>/<psi|psi> = sum |psi|^2 E_loc / sum |psi|^2 (to 1e-12)
    w = np.abs(psi) ** 2
    lhs = (np.conj(psi_sector) @ Hs @ psi_sector) / (np.conj(psi_sector) @ psi_sector)
    rhs = np.sum(w * e) / np.sum(w)
    assert abs(lhs.imag) < 1e-12
    assert abs(rhs - lhs) <= 1e-12 * max(1.0, abs(lhs))


def test_zero_variance_for_an_eigenvector():
    d = synth.config_inputs(1)
    K, nu, nd = d["K"], d["n_up"], d["n_dn"]
    Hs, idx = jw.sector_hamiltonian(K, nu, nd, d["h"], d["g"], d["e_core"])
    w, V = np.linalg.eigh(Hs.real)
    for level in (0, 3):
        v = V[:, level]
        keys = np.stack([_key_of_index(int(b)) for b in idx])
        logabs = np.log(np.abs(v))
        phase = np.where(v < 0, np.pi, 0.0)
        e = oracle.eloc_table(K, nu, nd, d["h"], d["g"], d["e_core"], keys, logabs, phase, keys, logabs, phase)
        # components that vanish by spin symmetry are 0/0 and carry no information
        big = np.abs(v) > 1e-6 * np.abs(v).max()
        assert big.sum() >= len(v) // 2
        assert np.abs(e[big] - w[level]).max() < 1e-10 * max(1.0, abs(w[level]))


def test_sample_aware_restriction_matches_masked_definition():
    """Section 3.4 item 4: only x' in the table contribute."""
    d = synth.config_inputs(1, K=5, n_up=2, n_dn=2)
    K, nu, nd = d["K"], d["n_up"], d["n_dn"]
    Hs, idx = jw.sector_hamiltonian(K, nu, nd, d["h"], d["g"], d["e_core"])
    Hs = Hs.real
    pos = {int(b): i for i, b in enumerate(idx)}
    rng = np.random.default_rng(11)
    keep = np.sort(rng.choice(len(d["keys"]), size=len(d["keys"]) // 3, replace=False))
    tk, tl, tp = d["keys"][keep], d["logabs"][keep], d["phase"][keep]
    psi_s = np.zeros(len(idx), complex)
    for k, l, p in zip(tk, tl, tp):
        psi_s[pos[_index_of_key(k)]] = np.exp(l + 1j * p)
    e = oracle.eloc_table(K, nu, nd, d["h"], d["g"], d["e_core"], tk, tl, tp, d["keys"], d["logabs"], d["phase"])
    for k in range(len(d["keys"])):
        x = pos[_index_of_key(d["keys"][k])]
        ref = (Hs[x] @ psi_s) / np.exp(d["logabs"][k] + 1j * d["phase"][k])
        assert abs(e[k] - ref) <= 1e-12 * max(1.0, abs(ref)) * np.abs(Hs).max()


# ------------------------------------------------------- structure / closed forms
@pytest.mark.parametrize("K,nu,nd", [(4, 2, 2), (24, 6, 6), (60, 20, 20), (10, 3, 4), (64, 1, 63), (3, 0, 3)])
def test_connection_count_closed_form(K, nu, nd):
    assert oracle.n_connections(K, nu, nd) == _closed_form_C(K, nu, nd)


def test_known_counts():
    assert oracle.n_connections(4, 2, 2) == 27
    assert oracle.n_connections(24, 6, 6) == 16471
    assert oracle.n_connections(60, 20, 20) == 938001


def test_hartree_fock_diagonal():
    """Textbook closed-shell HF energy: 2 sum_i h_ii + sum_ij [2 (ii|jj) - (ij|ji)]."""
    d = synth.config_inputs(2, n_unique=16)
    K, n = d["K"], d["n_up"]
    h, g = d["h"], d["g"]
    occ = range(n)
    ref = 2 * sum(h[i, i] for i in occ) + sum(2 * g[i, i, j, j] - g[i, j, j, i] for i in occ for j in occ)
    x = synth.hf_key(K, n, n)
    v, s = oracle.hxx(K, h, g, 0.0, x, x)
    assert s == 1 and abs(v - ref) < 1e-12 * abs(ref)


def test_hermiticity_and_conservation_on_config2_samples():
    d = synth.config_inputs(2, n_unique=8)
    K, nu, nd = d["K"], d["n_up"], d["n_dn"]
    even = np.uint64(0x5555555555555555)
    for x in d["keys"][:3]:
        xp, sign, exc, hv = oracle.connections(K, nu, nd, d["h"], d["g"], d["e_core"], x)
        for k in range(0, xp.shape[0], 7):
            y = xp[k]
            up = bin(int(y[0] & even)).count("1") + bin(int(y[1] & even)).count("1")
            dn = bin(int(y[0] & ~even)).count("1") + bin(int(y[1] & ~even)).count("1")
            assert (up, dn) == (nu, nd)
            back, _ = oracle.hxx(K, d["h"], d["g"], d["e_core"], y, x)
            assert abs(back - hv[k]) <= 1e-13 * max(1.0, abs(hv[k]))
            assert sign[k] in (1, -1)


def test_sort_table_matches_lexsort_and_searchsorted():
    d = synth.config_inputs(2, n_unique=2000, K=40, n_up=10, n_dn=9)
    keys = d["keys"].copy()
    keys[::3, 1] = np.uint64(1) << np.uint64(7)  # populate word 1 for some keys
    ko, lo, po, uniq = oracle.sort_table(keys, d["logabs"], d["phase"])
    order = np.lexsort((keys[:, 0], keys[:, 1]))
    assert (ko == keys[order]).all() and (lo == d["logabs"][order]).all()
    assert uniq == (len({(int(a), int(b)) for a, b in keys}) == len(keys))
    packed = [(int(b) << 64) | int(a) for a, b in ko]
    assert packed == sorted(packed)
    assert np.searchsorted(np.array(packed, dtype=object), packed[17]) == 17


def test_weighted_energy_equals_expanded_mean():
    """Eq. 6 with unique samples: weighting by counts = averaging the expanded list."""
    rng = np.random.default_rng(5)
    n = 50
    e = rng.normal(size=n) + 1j * rng.normal(size=n)
    c = rng.integers(1, 6, size=n).astype(np.uint32)
    out = oracle.energy(c, e)
    expanded = np.repeat(e, c)
    assert abs(out[0] - expanded.real.mean()) < 1e-13
    assert abs(out[1] - expanded.imag.mean()) < 1e-13
    assert out[2] == c.sum()
    assert abs(out[3] - expanded.real.var()) < 1e-12
