"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This module only draws random numbers and arranges them into integral tensors
and parameter vectors; it holds none of the method's arithmetic (no
Hamiltonian, no mapping, no circuit).  Both sides of every parity test take
their inputs from here and from nowhere else.

The paper's molecules (F2 and CH3F in STO-3G with a frozen core, Sec. 3.1 and
Sec. 3.2) and their integrals are not available, so every input is synthetic:

* one-body integrals ``h[p, q]`` over spatial orbitals, real symmetric;
* two-body integrals ``g[p, q, r, s]`` in chemist notation ``(pq|rs)``, real,
  with the 8-fold permutational symmetry of real molecular integrals;
* the nuclear-repulsion constant ``h0`` is 0 throughout.

Draw order (fixed, so a seed defines the tensors exactly):

* symmetric matrix: entries of the upper triangle including the diagonal, in
  row-major order ``p <= q``, then mirrored;
* 8-fold tensor: canonical quadruples with compound indices
  ``pq = p(p+1)/2 + q`` (``p >= q``), ``rs`` likewise, ``pq >= rs``, visited in
  increasing ``(pq, rs)``; each draw is copied into its 8 images.

For ``n`` qubits there are ``ns = ceil(n / 2)`` spatial orbitals; for odd ``n``
the last spatial orbital carries only an alpha spin orbital.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "n_spatial", "symmetric", "eightfold", "random_integrals",
    "scan_integrals", "warmstart_integrals", "uniform_theta", "batch_spec",
    "SCAN12_LAMBDAS", "WARM_LAMBDAS",
]

# Bond-stretch coordinates of the two scans (synthetic stand-ins for the
# paper's stretched geometries, Sec. 3.1 "Results for bond stretching").
SCAN12_LAMBDAS = np.linspace(0.8, 2.5, 20)
WARM_LAMBDAS = np.linspace(0.7, 3.0, 200)


def n_spatial(n_qubits: int) -> int:
    return (n_qubits + 1) // 2


def symmetric(rng: np.random.Generator, ns: int, std: float) -> np.ndarray:
    """Real symmetric ns x ns matrix, upper triangle ~ N(0, std^2)."""
    m = np.zeros((ns, ns))
    for p in range(ns):
        for q in range(p, ns):
            v = rng.normal(0.0, std)
            m[p, q] = v
            m[q, p] = v
    return m


def _canonical_quadruples(ns: int):
    pairs = [(p, q) for p in range(ns) for q in range(p + 1)]  # compound order
    for a, (p, q) in enumerate(pairs):
        for b in range(a + 1):
            r, s = pairs[b]
            yield p, q, r, s


def eightfold(rng: np.random.Generator, ns: int, std: float) -> np.ndarray:
    """Real (pq|rs) tensor with 8-fold symmetry, canonical entries ~ N(0, std^2)."""
    g = np.zeros((ns, ns, ns, ns))
    for p, q, r, s in _canonical_quadruples(ns):
        v = rng.normal(0.0, std)
        for (a, b, c, d) in ((p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                             (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)):
            g[a, b, c, d] = v
    return g


def random_integrals(n_qubits: int, seed: int):
    """Single-geometry integrals: h ~ N(0, 0.5^2) symmetric with diagonal - 1,
    g ~ N(0, 0.1^2) with 8-fold symmetry.  Returns (h0, h, g)."""
    rng = np.random.default_rng(seed)
    ns = n_spatial(n_qubits)
    h = symmetric(rng, ns, 0.5) - np.eye(ns)
    g = eightfold(rng, ns, 0.1)
    return 0.0, h, g


class _Family:
    """Integrals that vary smoothly with a stretch coordinate lam:
    h(lam) = sum_k H_k exp(-k lam), g(lam) = sum_k G_k exp(-k lam)."""

    def __init__(self, hs, gs):
        self.hs = hs
        self.gs = gs

    def __call__(self, lam: float):
        h = sum(hk * np.exp(-k * lam) for k, hk in enumerate(self.hs))
        g = sum(gk * np.exp(-k * lam) for k, gk in enumerate(self.gs))
        return 0.0, h, g


def scan_integrals(n_qubits: int, seed: int) -> _Family:
    """h(lam) = A_h + B_h e^-lam, g(lam) = A_g + B_g e^-lam.
    Draw order: A_h (sym 0.5, minus identity), B_h (sym 0.5), A_g, B_g (8-fold 0.1)."""
    rng = np.random.default_rng(seed)
    ns = n_spatial(n_qubits)
    a_h = symmetric(rng, ns, 0.5) - np.eye(ns)
    b_h = symmetric(rng, ns, 0.5)
    a_g = eightfold(rng, ns, 0.1)
    b_g = eightfold(rng, ns, 0.1)
    return _Family([a_h, b_h], [a_g, b_g])


def warmstart_integrals(n_qubits: int, seed: int) -> _Family:
    """h, g = A + B e^-lam + C e^-2lam.  Draw order: A_h, B_h, C_h, A_g, B_g, C_g."""
    rng = np.random.default_rng(seed)
    ns = n_spatial(n_qubits)
    a_h = symmetric(rng, ns, 0.5) - np.eye(ns)
    b_h = symmetric(rng, ns, 0.5)
    c_h = symmetric(rng, ns, 0.5)
    a_g = eightfold(rng, ns, 0.1)
    b_g = eightfold(rng, ns, 0.1)
    c_g = eightfold(rng, ns, 0.1)
    return _Family([a_h, b_h, c_h], [a_g, b_g, c_g])


def uniform_theta(seed: int, m: int, lo: float = -0.1, hi: float = 0.1) -> np.ndarray:
    return np.random.default_rng(seed).uniform(lo, hi, size=m)


def batch_spec(n_states: int = 512, seed: int = 3, n_min: int = 12, n_max: int = 20):
    """Qubit counts of the batched workload: n_i ~ U{n_min..n_max}, electrons
    floor(n_i / 2); state i draws its integrals and amplitudes from seed
    30000 + i.  Returns a list of (n_qubits, n_electrons, seed_i)."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_min, n_max + 1, size=n_states)
    return [(int(n), int(n) // 2, 30000 + i) for i, n in enumerate(ns)]
