"""Literal brute force of Eq. 9 through the Jordan-Wigner mapping (tests only).

Builds every annihilator as a sparse ``2^N x 2^N`` matrix from Pauli matrices,
``a_p = Z_0 ... Z_{p-1} (X_p + i Y_p)/2``, assembles

    H = E_core + sum_pq h^p_q a+_p a_q + 1/2 sum_pqrs g^{pq}_{rs} a+_p a+_q a_r a_s

term by term with ``g^{pq}_{rs} = <pq|sr> = (i_p i_s | i_q i_r)`` (spin-diagonal),
and restricts it to a particle/spin sector.  Basis index ``b = sum_p x_p 2^p``:
bit ``p`` of the index is the occupation of spin orbital ``p``.  It shares no
code with the oracle and uses no Slater-Condon rule.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

_I = sp.identity(2, format="csr", dtype=np.complex128)
_X = sp.csr_matrix(np.array([[0, 1], [1, 0]], dtype=np.complex128))
_Y = sp.csr_matrix(np.array([[0, -1j], [1j, 0]], dtype=np.complex128))
_Z = sp.csr_matrix(np.array([[1, 0], [0, -1]], dtype=np.complex128))


def annihilator(p: int, N: int) -> sp.csr_matrix:
    op = sp.identity(1, format="csr", dtype=np.complex128)
    for q in reversed(range(N)):  # leftmost Kronecker factor = most significant bit
        if q < p:
            f = _Z
        elif q == p:
            f = (_X + 1j * _Y) * 0.5
        else:
            f = _I
        op = sp.kron(op, f, format="csr")
    return op


def hamiltonian(K: int, h: np.ndarray, g: np.ndarray, e_core: float = 0.0) -> sp.csr_matrix:
    N = 2 * K
    a = [annihilator(p, N) for p in range(N)]
    ad = [m.conj().T.tocsr() for m in a]
    dim = 1 << N
    H = sp.identity(dim, format="csr", dtype=np.complex128) * e_core
    spin = [p & 1 for p in range(N)]
    orb = [p >> 1 for p in range(N)]
    for p in range(N):
        for q in range(N):
            if spin[p] == spin[q] and h[orb[p], orb[q]] != 0.0:
                H = H + h[orb[p], orb[q]] * (ad[p] @ a[q])
    for p in range(N):
        for q in range(N):
            pq = ad[p] @ ad[q]
            if pq.nnz == 0:
                continue
            for r in range(N):
                for s in range(N):
                    # g^{pq}_{rs} = (p s | q r): pairs (p, s) and (q, r) share a spin
                    if spin[p] != spin[s] or spin[q] != spin[r]:
                        continue
                    c = g[orb[p], orb[s], orb[q], orb[r]]
                    if c == 0.0:
                        continue
                    H = H + (0.5 * c) * (pq @ (a[r] @ a[s]))
    return H.tocsr()


def sector_indices(K: int, n_up: int, n_dn: int) -> np.ndarray:
    """Basis indices of the (n_up, n_dn) sector, ascending."""
    N = 2 * K
    idx = []
    for b in range(1 << N):
        up = sum((b >> (2 * i)) & 1 for i in range(K))
        dn = sum((b >> (2 * i + 1)) & 1 for i in range(K))
        if up == n_up and dn == n_dn:
            idx.append(b)
    return np.array(idx, dtype=np.int64)


def sector_hamiltonian(K, n_up, n_dn, h, g, e_core=0.0):
    """Dense sector block ``H[b', b] = <b'|H|b>`` and the sector's basis indices."""
    H = hamiltonian(K, h, g, e_core)
    idx = sector_indices(K, n_up, n_dn)
    Hs = H[idx][:, idx].toarray()
    return Hs, idx


def index_to_key(b: int) -> np.ndarray:
    return np.array([b & 0xFFFFFFFFFFFFFFFF, b >> 64], dtype=np.uint64)
