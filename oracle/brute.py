"""Full Fock-space matrices from the definition of the ladder operators
(test infrastructure only; n <= 8).

a_P^dag |b> = (-1)^(sum_{q<P} b_q) |b + e_P> if b_P = 0, else 0 — the
Jordan-Wigner ordering of spin orbitals (Sec. 2.1.1), with bit P of the
basis index the occupation of spin orbital P.  Everything here is built by
looping over basis states, so it shares no construction with ``fermion``
(sector strings, operator caches) or ``pauli`` (Pauli algebra), and pins both.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg
import scipy.sparse


def creation(n: int, P: int):
    """a_P^dag as a sparse 2^n x 2^n matrix, one basis state at a time."""
    dim = 1 << n
    rows, cols, vals = [], [], []
    for b in range(dim):
        if (b >> P) & 1:
            continue
        sign = -1.0 if bin(b & ((1 << P) - 1)).count("1") % 2 else 1.0
        rows.append(b | (1 << P))
        cols.append(b)
        vals.append(sign)
    return scipy.sparse.csr_matrix((vals, (rows, cols)), shape=(dim, dim))


def ladder(n: int):
    cr = [creation(n, P) for P in range(n)]
    an = [c.T.tocsr() for c in cr]
    return cr, an


def hamiltonian(n: int, h0, h, g) -> np.ndarray:
    """Eq. 2 written out on spin orbitals:
    H = h0 + sum_PQ h_PQ a_P^dag a_Q + sum_PQRS h_PQRS a_P^dag a_Q^dag a_R a_S,
    h_PQ = h_pq delta(s_P, s_Q),
    h_PQRS = 1/2 (ps|qr) delta(s_P, s_S) delta(s_Q, s_R)."""
    cr, an = ladder(n)
    dim = 1 << n
    H = h0 * scipy.sparse.identity(dim, format="csr")
    sp = lambda P: P // 2
    for P in range(n):
        for Q in range(n):
            if P % 2 == Q % 2:
                H += h[sp(P), sp(Q)] * (cr[P] @ an[Q])
    for P in range(n):
        for Q in range(n):
            for R in range(n):
                for S in range(n):
                    if P % 2 != S % 2 or Q % 2 != R % 2:
                        continue
                    v = 0.5 * g[sp(P), sp(S), sp(Q), sp(R)]
                    if v != 0.0:
                        H += v * (cr[P] @ cr[Q] @ an[R] @ an[S])
    return H.toarray()


def number_ops(n: int):
    cr, an = ladder(n)
    N = sum((cr[P] @ an[P]).toarray() for P in range(n))
    Sz = sum((0.5 if P % 2 == 0 else -0.5) * (cr[P] @ an[P]).toarray() for P in range(n))
    return N, Sz


def excitation_generator(n: int, exc) -> np.ndarray:
    """T - T^dag for a single (i, a) or double (i, j, a, b) excitation."""
    cr, an = ladder(n)
    if len(exc) == 2:
        i, a = exc
        T = cr[a] @ an[i]
    else:
        i, j, a, b = exc
        T = cr[a] @ cr[b] @ an[j] @ an[i]
    return (T - T.T).toarray()


def excitation_unitary(n: int, exc, theta: float) -> np.ndarray:
    return scipy.linalg.expm(theta * excitation_generator(n, exc))


def sector_indices(n: int, n_alpha: int, n_beta: int) -> np.ndarray:
    idx = []
    for b in range(1 << n):
        na = sum((b >> q) & 1 for q in range(0, n, 2))
        nb = sum((b >> q) & 1 for q in range(1, n, 2))
        if na == n_alpha and nb == n_beta:
            idx.append(b)
    return np.array(idx, dtype=np.int64)
