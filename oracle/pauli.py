"""Dense-Pauli oracle mode (test infrastructure only; n <= 14).

An independent Jordan-Wigner construction (Sec. 2.1.1: the fermionic
Hamiltonian of Eq. 2 is mapped to qubit operators) done with Hermitian
Pauli-string algebra, and a statevector evolution by Pauli rotations
exp(-i phi/2 P) acting on the full 2^n vector.

A Pauli string is keyed by two bit masks (x, z): on qubit q the factor is
I (x_q=0, z_q=0), X (1, 0), Y (1, 1) or Z (0, 1).  A Pauli sum is a dict
{(x, z): complex coefficient}.  Products are taken qubit by qubit from the
single-qubit multiplication table, and strings act on basis states qubit by
qubit from the 2x2 matrices, so no phase identity is shared with the HIP
path's folded representation.
"""
from __future__ import annotations

from collections import defaultdict
import math

import numpy as np

# single-qubit Paulis as (x, z) bits: I=(0,0) X=(1,0) Y=(1,1) Z=(0,1)
_NAME = {(0, 0): "I", (1, 0): "X", (1, 1): "Y", (0, 1): "Z"}
_BITS = {v: k for k, v in _NAME.items()}
# products a*b = phase * c
_TABLE = {
    ("I", "I"): (1, "I"), ("I", "X"): (1, "X"), ("I", "Y"): (1, "Y"), ("I", "Z"): (1, "Z"),
    ("X", "I"): (1, "X"), ("Y", "I"): (1, "Y"), ("Z", "I"): (1, "Z"),
    ("X", "X"): (1, "I"), ("Y", "Y"): (1, "I"), ("Z", "Z"): (1, "I"),
    ("X", "Y"): (1j, "Z"), ("Y", "X"): (-1j, "Z"),
    ("Y", "Z"): (1j, "X"), ("Z", "Y"): (-1j, "X"),
    ("Z", "X"): (1j, "Y"), ("X", "Z"): (-1j, "Y"),
}
# action on a basis bit: P|v> = phase |v'>
_ACT = {
    "I": {0: (1, 0), 1: (1, 1)},
    "X": {0: (1, 1), 1: (1, 0)},
    "Y": {0: (1j, 1), 1: (-1j, 0)},
    "Z": {0: (1, 0), 1: (-1, 1)},
}


def _letter(x, z, q):
    return _NAME[((x >> q) & 1, (z >> q) & 1)]


def string_product(a, b, n):
    (xa, za), (xb, zb) = a, b
    phase = 1
    x = z = 0
    for q in range(n):
        ph, c = _TABLE[(_letter(xa, za, q), _letter(xb, zb, q))]
        phase *= ph
        bx, bz = _BITS[c]
        x |= bx << q
        z |= bz << q
    return phase, (x, z)


def sum_product(A, B, n):
    out = defaultdict(complex)
    for ka, ca in A.items():
        for kb, cb in B.items():
            ph, k = string_product(ka, kb, n)
            out[k] += ph * ca * cb
    return out


def ladder(n, P, dagger, mapping="jw"):
    """Jordan-Wigner: a_P^dag = Z_0..Z_{P-1} (X_P - iY_P)/2,
    a_P = Z_0..Z_{P-1} (X_P + iY_P)/2.  Bravyi-Kitaev: see bk_ladder."""
    if mapping == "bk":
        return bk_ladder(n, P, dagger)
    chain = (1 << P) - 1
    s = -1j if dagger else 1j
    return {(1 << P, chain): 0.5, ((1 << P), chain | (1 << P)): 0.5 * s}


# --- Bravyi-Kitaev (Sec. 2.1.1 names the mapping) --------------------------
# Qubit j stores the parity of the orbitals of its Fenwick-tree node,
# j & (j + 1) .. j.  With the published sets of the transformation (update
# set U: nodes above j that also store n_j; parity set P: nodes whose
# parities add up to n_0 + .. + n_{j-1}; flip set F: the nodes below j inside
# j's own range, so that n_j = b_j + sum_F b; remainder R = P minus F):
#   a_j^dag = 1/2 X_U (X_j Z_P - i Y_j Z_R),  a_j = 1/2 X_U (X_j Z_P + i Y_j Z_R).

def bk_sets(n, j):
    """(U, P, F, R) of orbital j as bit masks."""
    U = 0
    k = j | (j + 1)
    while k < n:
        U |= 1 << k
        k = k | (k + 1)
    P = 0
    k = j - 1
    while k >= 0:
        P |= 1 << k
        k = (k & (k + 1)) - 1
    F = 0
    lo = j & (j + 1)
    k = j - 1
    while k >= lo:
        F |= 1 << k
        k = (k & (k + 1)) - 1
    return U, P, F, P & ~F


def bk_encode(n, occ):
    """Qubit register of the occupation bits occ."""
    b = 0
    for j in range(n):
        par = 0
        for k in range(j & (j + 1), j + 1):
            par ^= (occ >> k) & 1
        b |= par << j
    return b


def bk_ladder(n, j, dagger):
    U, P, _, R = bk_sets(n, j)
    e = 1 << j
    s = -1j if dagger else 1j
    # X on U and j with Z on P; X on U, Y on j (x = z = 1 there), Z on R
    return {(U | e, P): 0.5, (U | e, R | e): 0.5 * s}


def _clean(S, tol=1e-12):
    return {k: v for k, v in S.items() if abs(v) > tol}


def jw_hamiltonian(n, h0, h, g, tol=1e-12, mapping="jw"):
    """Qubit form of Eq. 2 (chemist integrals, factor 1/2; see fermion.py)
    under the Jordan-Wigner (default) or Bravyi-Kitaev mapping."""
    cr = [ladder(n, P, True, mapping) for P in range(n)]
    an = [ladder(n, P, False, mapping) for P in range(n)]
    H = defaultdict(complex)
    H[(0, 0)] += h0
    sp = lambda P: P // 2
    one = {}
    for P in range(n):
        for Q in range(n):
            if P % 2 == Q % 2 and h[sp(P), sp(Q)] != 0.0:
                one[(P, Q)] = sum_product(cr[P], an[Q], n)
                for k, v in one[(P, Q)].items():
                    H[k] += h[sp(P), sp(Q)] * v
    for P in range(n):
        for R in range(n):
            if P == R:
                continue
            left = sum_product(cr[P], cr[R], n)
            for S in range(n):
                if S % 2 != R % 2:
                    continue
                for Q in range(n):
                    if Q % 2 != P % 2 or Q == S:
                        continue
                    v = 0.5 * g[sp(P), sp(Q), sp(R), sp(S)]
                    if v == 0.0:
                        continue
                    term = sum_product(left, sum_product(an[S], an[Q], n), n)
                    for k, c in term.items():
                        H[k] += v * c
    return _clean(H, tol)


def apply_string(key, psi, n):
    """P |psi> for one Pauli string, from the single-qubit 2x2 actions."""
    x, z = key
    dim = 1 << n
    b = np.arange(dim, dtype=np.int64)
    phase = np.ones(dim, dtype=np.complex128)
    tgt = b.copy()
    for q in range(n):
        L = _letter(x, z, q)
        if L == "I":
            continue
        bit = (b >> q) & 1
        ph0, v0 = _ACT[L][0]
        ph1, v1 = _ACT[L][1]
        phase *= np.where(bit == 0, ph0, ph1)
        newbit = np.where(bit == 0, v0, v1)
        tgt = (tgt & ~(1 << q)) | (newbit << q)
    out = np.zeros_like(psi)
    out[tgt] = phase * psi
    return out


def apply_sum(S, psi, n):
    out = np.zeros_like(psi)
    for k, c in S.items():
        out += c * apply_string(k, psi, n)
    return out


def energy(S, psi, n) -> float:
    return float(np.real(np.vdot(psi, apply_sum(S, psi, n))))


def matrix(S, n):
    dim = 1 << n
    m = np.zeros((dim, dim), dtype=np.complex128)
    for c in range(dim):
        e = np.zeros(dim, dtype=np.complex128)
        e[c] = 1.0
        m[:, c] = apply_sum(S, e, n)
    return m


def excitation_generator(n, exc, mapping="jw"):
    """T - T^dag as a Pauli sum (T = a_a^dag a_i or a_a^dag a_b^dag a_j a_i)."""
    cr = lambda P: ladder(n, P, True, mapping)
    an = lambda P: ladder(n, P, False, mapping)
    if len(exc) == 2:
        i, a = exc
        T = sum_product(cr(a), an(i), n)
        Td = sum_product(cr(i), an(a), n)
    else:
        i, j, a, b = exc
        T = sum_product(sum_product(cr(a), cr(b), n), sum_product(an(j), an(i), n), n)
        Td = sum_product(sum_product(cr(i), cr(j), n), sum_product(an(b), an(a), n), n)
    G = defaultdict(complex)
    for k, v in T.items():
        G[k] += v
    for k, v in Td.items():
        G[k] -= v
    return _clean(G)


def excitation_rotations(n, exc, mapping="jw"):
    """T - T^dag = i sum_k b_k P_k (b_k real, commuting P_k), hence
    exp(theta (T - T^dag)) = prod_k exp(-i (phi_k / 2) P_k) with phi_k = -2 b_k theta.
    Returns [(x, z, scale_k)] with phi_k = scale_k * theta."""
    out = []
    for (x, z), c in sorted(excitation_generator(n, exc, mapping).items()):
        if abs(c.real) > 1e-14:
            raise AssertionError("generator coefficient not imaginary")
        out.append((x, z, -2.0 * c.imag))
    return out


def apply_rotation(psi, n, key, phi):
    """exp(-i phi/2 P) psi = cos(phi/2) psi - i sin(phi/2) P psi."""
    return math.cos(phi / 2) * psi - 1j * math.sin(phi / 2) * apply_string(key, psi, n)


def prepare(n, n_electrons, excs, theta, mapping="jw"):
    psi = np.zeros(1 << n, dtype=np.complex128)
    ref = (1 << n_electrons) - 1
    psi[bk_encode(n, ref) if mapping == "bk" else ref] = 1.0
    for exc, t in zip(excs, theta):
        for x, z, sc in excitation_rotations(n, exc, mapping):
            psi = apply_rotation(psi, n, (x, z), sc * float(t))
    return psi


def folded_terms(S):
    """Terms in the folded real form c' X^x Z^z (c' = c i^{#Y}), as used at
    the library boundary.  Returns {(x, z): real c'}; raises if c' is not real."""
    out = {}
    for (x, z), c in S.items():
        y = bin(x & z).count("1")
        f = c * (1j ** y)
        if abs(f.imag) > 1e-12:
            raise AssertionError("folded coefficient not real")
        out[(x, z)] = f.real
    return out
