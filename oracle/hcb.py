"""Hard-core-boson oracle for the pUCCD ansatz (test infrastructure only; see
the package docstring).

pUCCD (Sec. 2.1, the ansatz list: "pUCCD") keeps only the double
excitations that move both electrons of one spatial orbital into another.
Such a state stays in the seniority-zero space (every spatial orbital doubly
occupied or empty), where a pair behaves as a hard-core boson: qubit p is
spatial orbital p, bit p = 1 when the pair is present, half the qubits of
the Jordan-Wigner form.

Hamiltonian: Eq. 2 (read with chemist integrals and the factor 1/2, as in
``fermion``) projected onto the seniority-zero space.  For a pair set O the
Slater-Condon rule gives the diagonal

  E_O = h0 + sum_{p in O} (2 h_pp + (pp|pp)) + sum_{p != q in O} [2 (pp|qq) - (pq|qp)],

and moving the pair on q to an empty p is the double excitation
(q alpha, q beta) -> (p alpha, p beta) with matrix element <pa pb||qa qb> =
(pq|pq); its ladder-operator sign is +1 because the orbitals below each
operator hold whole pairs.  One-electron moves leave the space and drop out.
So, with N_p the pair number and b_p the pair annihilator,

  H = h0 + sum_p e_p N_p + sum_{p<q} w_pq N_p N_q + sum_{p != q} v_pq b_p^dag b_q,
  e_p = 2 h_pp + (pp|pp),  w_pq = 2 [2 (pp|qq) - (pq|qp)],  v_pq = (pq|pq).

Ansatz: U = prod exp(theta_k (b_a^dag b_i - b_i^dag b_a)) over occupied pairs
i and empty orbitals a of the reference (a outer, i inner, ascending; a
reading, matching the UCCSD doubles' order); each factor is a Givens
rotation with T|D> = +|E>.
"""
from __future__ import annotations

from itertools import combinations
import math

import numpy as np


def coefficients(h0, h, g):
    """(h0, e[p], w[p, q] (p < q, else 0), v[p, q] (p != q, else 0))."""
    ns = h.shape[0]
    e = np.array([2.0 * h[p, p] + g[p, p, p, p] for p in range(ns)])
    w = np.zeros((ns, ns))
    v = np.zeros((ns, ns))
    for p in range(ns):
        for q in range(ns):
            if p < q:
                w[p, q] = 2.0 * (2.0 * g[p, p, q, q] - g[p, q, q, p])
            if p != q:
                v[p, q] = g[p, q, p, q]
    return float(h0), e, w, v


class Space:
    """Pair-occupation patterns of n_orb orbitals holding n_pairs pairs."""

    def __init__(self, n_orb: int, n_pairs: int):
        if not (1 <= n_orb <= 30) or not (0 <= n_pairs <= n_orb):
            raise ValueError("sizes out of range")
        self.n = n_orb
        self.np = n_pairs
        self.bits = np.array(sorted(sum(1 << p for p in c) for c in combinations(range(n_orb), n_pairs)),
                             dtype=np.int64)
        self.index = {int(b): k for k, b in enumerate(self.bits)}
        self.ndet = self.bits.size
        self.hf_bits = (1 << n_pairs) - 1

    def hf(self) -> np.ndarray:
        psi = np.zeros(self.ndet, dtype=np.complex128)
        psi[self.index[self.hf_bits]] = 1.0
        return psi

    def to_statevector(self, psi):
        full = np.zeros(1 << self.n, dtype=np.complex128)
        full[self.bits] = psi
        return full


def hamiltonian_matrix(space: Space, h0, h, g) -> np.ndarray:
    """Dense H on the space, entry by entry from the definitions above."""
    c0, e, w, v = coefficients(h0, h, g)
    n = space.n
    m = np.zeros((space.ndet, space.ndet))
    for k, b in enumerate(space.bits):
        occ = [p for p in range(n) if (b >> p) & 1]
        m[k, k] = c0 + sum(e[p] for p in occ) + sum(w[p, q] for p in occ for q in occ if p < q)
        for q in occ:
            for p in range(n):
                if (b >> p) & 1:
                    continue
                t = int(b) ^ (1 << q) ^ (1 << p)
                m[space.index[t], k] += v[p, q]
    return m


def puccd_excitations(n_orb: int, n_pairs: int):
    """(i, a) pairs, a outer and i inner, ascending."""
    return [(i, a) for a in range(n_pairs, n_orb) for i in range(n_pairs)]


def apply_pair(space: Space, psi, exc, theta):
    """psi <- exp(theta (b_a^dag b_i - b_i^dag b_a)) psi."""
    i, a = exc
    c, s = math.cos(theta), math.sin(theta)
    out = psi.copy()
    for k, b in enumerate(space.bits):
        if ((b >> i) & 1) and not ((b >> a) & 1):
            kk = space.index[int(b) ^ (1 << i) ^ (1 << a)]
            out[k] = c * psi[k] - s * psi[kk]
            out[kk] = c * psi[kk] + s * psi[k]
    return out


class Problem:
    """pUCCD on the hard-core-boson space."""

    def __init__(self, n_orb: int, n_pairs: int, h0, h, g, excs=None):
        self.space = Space(n_orb, n_pairs)
        self.H = hamiltonian_matrix(self.space, h0, h, g)
        self.excs = puccd_excitations(n_orb, n_pairs) if excs is None else list(excs)

    @property
    def n_params(self):
        return len(self.excs)

    def state(self, theta):
        psi = self.space.hf()
        for exc, t in zip(self.excs, theta):
            psi = apply_pair(self.space, psi, exc, float(t))
        return psi

    def energy(self, theta) -> float:
        psi = self.state(theta)
        return float(np.real(np.vdot(psi, self.H @ psi)))

    def grad_shift(self, theta):
        """Four-term shift rule (frequencies {1, 2}; see fermion.Problem)."""
        theta = np.asarray(theta, dtype=np.float64)
        c2 = (math.sqrt(2.0) - 1.0) / 2.0
        out = []
        for j in range(theta.size):
            def e(d):
                t = theta.copy()
                t[j] += d
                return self.energy(t)
            out.append((e(math.pi / 4) - e(-math.pi / 4)) - c2 * (e(math.pi / 2) - e(-math.pi / 2)))
        return np.array(out)

    def ground(self) -> float:
        return float(np.linalg.eigvalsh(self.H)[0])
