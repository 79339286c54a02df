"""CI-space oracle (test infrastructure only; see the package docstring).

Representation
--------------
Qubit / spin-orbital ``q`` is spatial orbital ``q // 2`` with spin ``q % 2``
(0 = alpha, 1 = beta).  For odd qubit counts the last spatial orbital has an
alpha spin orbital only.  Bit ``q`` of a basis-state index is the occupation
of spin orbital ``q`` (Jordan-Wigner ordering, Sec. 2.1.1).

The wavefunction lives in the (N, S_z) sector reached from Hartree-Fock: all
determinants with ``n_alpha = ceil(n_e / 2)`` alpha and ``n_beta = floor(n_e / 2)``
beta electrons.  Every operator the method applies (the Hamiltonian, Eq. 2,
and the UCCSD generators, Sec. 2.1.2) conserves both counts, so nothing
outside the sector is ever populated.  ``Space.bits`` holds the full
statevector index of each sector determinant, so results map one-to-one onto
a 2^n statevector.

Readings of the paper used here (where it is silent or garbled)
---------------------------------------------------------------
* Eq. 2 is taken with chemist integrals and a factor 1/2:
  h_{ijkl} a_i^dag a_j^dag a_k a_l with h_{ijkl} = 1/2 (il|jk) for
  sigma_i = sigma_l, sigma_j = sigma_k, else 0.
* h0 is an input (0 for every synthetic workload).
* UCCSD (Sec. 2.1.2): singles a_a^dag a_i, doubles a_a^dag a_b^dag a_j a_i with
  i < j occupied, a < b virtual, spin-conserving; one Trotter step; order:
  all singles (a outer, i inner), then doubles ((a, b) outer, (i, j) inner),
  ascending; U = U_M ... U_1 with U_j = exp(theta_j (T_j - T_j^dag)).
"""
from __future__ import annotations

from itertools import combinations
import math

import numpy as np
import scipy.linalg
import scipy.optimize
import scipy.sparse.linalg


def _popcount(a):
    return np.bitwise_count(a).astype(np.int64)


def _spread(strings: np.ndarray, spin: int) -> np.ndarray:
    """Place bit p of an orbital string at statevector bit 2p + spin."""
    out = np.zeros_like(strings)
    for p in range(64 // 2):
        out |= ((strings >> p) & 1) << (2 * p + spin)
    return out


def _strings(norb: int, nel: int) -> np.ndarray:
    return np.array([sum(1 << p for p in c) for c in combinations(range(norb), nel)],
                    dtype=np.int64)


class Space:
    """The (N, S_z) determinant space of n qubits and n_e electrons."""

    def __init__(self, n_qubits: int, n_electrons: int):
        if not (1 <= n_qubits <= 40):
            raise ValueError("n_qubits out of range")
        if not (0 <= n_electrons <= n_qubits):
            raise ValueError("n_electrons out of range")
        self.n = n_qubits
        self.ne = n_electrons
        self.norb_a = (n_qubits + 1) // 2
        self.norb_b = n_qubits // 2
        self.na = (n_electrons + 1) // 2
        self.nb = n_electrons // 2
        if self.na > self.norb_a or self.nb > self.norb_b:
            raise ValueError("electron count does not fit the spin orbitals")
        a = _spread(_strings(self.norb_a, self.na), 0)
        b = _spread(_strings(self.norb_b, self.nb), 1)
        self.bits = (a[:, None] | b[None, :]).ravel()
        self.ndet = self.bits.size
        self._order = np.argsort(self.bits, kind="stable")
        self._sorted = self.bits[self._order]
        self.hf_bits = (1 << n_electrons) - 1
        self._cache = {}

    def index_of(self, bits: np.ndarray) -> np.ndarray:
        pos = np.searchsorted(self._sorted, bits)
        pos = np.minimum(pos, self.ndet - 1)
        if not np.array_equal(self._sorted[pos], bits):
            raise AssertionError("determinant outside the sector")
        return self._order[pos]

    def hf(self) -> np.ndarray:
        psi = np.zeros(self.ndet, dtype=np.complex128)
        psi[self.index_of(np.array([self.hf_bits]))[0]] = 1.0
        return psi

    def to_statevector(self, psi: np.ndarray) -> np.ndarray:
        full = np.zeros(1 << self.n, dtype=np.complex128)
        full[self.bits] = psi
        return full

    # -- ladder-operator strings -------------------------------------------
    def op_string(self, ops):
        """Action of a product of ladder operators on every sector determinant.

        ``ops`` is written left to right, e.g. ((a, +1), (i, -1)) for
        a_a^dag a_i; it is applied right to left.  Each operator on orbital p
        contributes (-1)^(number of occupied orbitals below p) in the state it
        acts on (Jordan-Wigner ordering).  Returns (source indices, target
        indices, signs) for the determinants it does not annihilate; the
        target must lie in the sector.
        """
        key = tuple(ops)
        if key in self._cache:
            return self._cache[key]
        state = self.bits.copy()
        sign = np.ones(self.ndet, dtype=np.int64)
        alive = np.ones(self.ndet, dtype=bool)
        for p, kind in reversed(ops):
            occ = (state >> p) & 1
            alive &= (occ == 0) if kind > 0 else (occ == 1)
            below = state & ((1 << p) - 1)
            sign *= 1 - 2 * (_popcount(below) & 1)
            state = state ^ (1 << p)
        src = np.nonzero(alive)[0]
        dst = self.index_of(state[alive]) if src.size else src
        out = (src, dst, sign[alive].astype(np.float64))
        self._cache[key] = out
        return out


# --------------------------------------------------------------------------
# Ansatz (Sec. 2.1.2)
# --------------------------------------------------------------------------

def uccsd_excitations(n_qubits: int, n_electrons: int):
    """UCCSD excitation list in the fixed application order (see module doc)."""
    occ = list(range(n_electrons))
    virt = list(range(n_electrons, n_qubits))
    singles = [(i, a) for a in virt for i in occ if i % 2 == a % 2]
    doubles = [(i, j, a, b) for (a, b) in combinations(virt, 2)
               for (i, j) in combinations(occ, 2)
               if (i % 2) + (j % 2) == (a % 2) + (b % 2)]
    return singles + doubles


def kupccgsd_layer(n_qubits: int):
    """One k-UpCCGSD layer (Sec. 2.1, ansatz list), in application order
    (reading): generalised singles (p, q) = a_q^dag a_p for p < q of equal
    spin (q outer, p inner), then pair doubles (2p, 2p+1, 2q, 2q+1) =
    a_2q^dag a_2q+1^dag a_2p+1 a_2p for spatial p < q with both spin
    orbitals (q outer, p inner)."""
    singles = [(p, q) for q in range(n_qubits) for p in range(q) if p % 2 == q % 2]
    npair = n_qubits // 2
    doubles = [(2 * p, 2 * p + 1, 2 * q, 2 * q + 1) for q in range(npair) for p in range(q)]
    return singles + doubles


def kupccgsd_excitations(n_qubits: int, k: int):
    """k layers, each with its own angles."""
    return kupccgsd_layer(n_qubits) * k


def trotter_expand(excs, theta, steps: int):
    """UCC with `steps` Trotter steps (reading of the UCCSD depth): the product
    over excs with angles theta / steps, repeated steps times.  Returns the
    expanded excitation list and angles."""
    theta = np.asarray(theta, dtype=np.float64)
    return list(excs) * steps, np.tile(theta / steps, steps)


def excitation_ops(exc):
    """T of an excitation as a ladder-operator string (left to right)."""
    if len(exc) == 2:
        i, a = exc
        return ((a, +1), (i, -1))
    i, j, a, b = exc
    return ((a, +1), (b, +1), (j, -1), (i, -1))


def apply_excitation(space: Space, psi: np.ndarray, exc, theta: float) -> np.ndarray:
    """psi <- exp(theta (T - T^dag)) psi, in closed form.

    T maps each determinant D it does not annihilate to s_D E (s_D = +-1) and
    T^dag maps E back to s_D D, so on each such pair T - T^dag is the 2x2
    generator [[0, -s], [s, 0]] in the (D, E) basis and the exponential is a
    Givens rotation by theta.  Determinants outside all pairs are annihilated
    by both T and T^dag and stay unchanged.
    """
    src, dst, s = space.op_string(excitation_ops(exc))
    c, sn = math.cos(theta), math.sin(theta)
    pd = psi[src].copy()
    pe = psi[dst].copy()
    out = psi.copy()
    out[src] = c * pd - s * sn * pe
    out[dst] = c * pe + s * sn * pd
    return out


def prepare(space: Space, excs, theta) -> np.ndarray:
    """U_M ... U_1 |HF> (Eq. 1's U(theta)|0> with |0> the HF determinant)."""
    psi = space.hf()
    for exc, t in zip(excs, theta):
        psi = apply_excitation(space, psi, exc, float(t))
    return psi


# --------------------------------------------------------------------------
# Hamiltonian (Eq. 2)
# --------------------------------------------------------------------------

class Hamiltonian:
    """H = h0 + sum_PQ h_pq a_P^dag a_Q + 1/2 sum (pq|rs) a_P^dag a_R^dag a_S a_Q
    over spin orbitals P=(p,s), Q=(q,s), R=(r,t), S=(s',t) (Eq. 2, read with
    chemist integrals and the factor 1/2).

    sigma = H psi uses the exact rearrangement
      a_P^dag a_R^dag a_S a_Q = E_PQ E_RS - delta_QR a_P^dag a_S,
    with E_PQ = a_P^dag a_Q, so that
      sigma = h0 psi + sum_PQ E_PQ [k_PQ psi + 1/2 sum_RS (pq|rs) E_RS psi],
      k_PQ = h_pq - 1/2 sum_{R same spin as P} (pr|rq).
    """

    def __init__(self, space: Space, h0: float, h: np.ndarray, g: np.ndarray):
        self.space = space
        self.h0 = float(h0)
        n = space.n
        ns = (n + 1) // 2
        if h.shape != (ns, ns) or g.shape != (ns,) * 4:
            raise ValueError("integral shapes do not match the qubit count")
        self.pairs = [(P, Q) for P in range(n) for Q in range(n) if P % 2 == Q % 2]
        pq = [(P // 2, Q // 2) for P, Q in self.pairs]
        self.V = np.array([[g[p, q, r, s] for (r, s) in pq] for (p, q) in pq])
        self.k = np.empty(len(self.pairs))
        for idx, (P, Q) in enumerate(self.pairs):
            p, q = P // 2, Q // 2
            same = [R // 2 for R in range(n) if R % 2 == P % 2]
            self.k[idx] = h[p, q] - 0.5 * sum(g[p, r, r, q] for r in same)
        self.ops = [space.op_string(((P, +1), (Q, -1))) for P, Q in self.pairs]

    def _E(self, idx, vec):
        src, dst, s = self.ops[idx]
        out = np.zeros_like(vec)
        out[dst] = s * vec[src]
        return out

    def apply(self, psi: np.ndarray) -> np.ndarray:
        D = np.stack([self._E(i, psi) for i in range(len(self.pairs))])
        G = self.V @ D
        sigma = self.h0 * psi
        for i in range(len(self.pairs)):
            src, dst, s = self.ops[i]
            w = self.k[i] * psi + 0.5 * G[i]
            sigma[dst] += s * w[src]
        return sigma

    def expectation(self, psi: np.ndarray) -> float:
        return float(np.real(np.vdot(psi, self.apply(psi))))

    def matrix(self) -> np.ndarray:
        """Dense sector matrix (columns = H applied to unit vectors)."""
        nd = self.space.ndet
        m = np.empty((nd, nd), dtype=np.complex128)
        e = np.zeros(nd, dtype=np.complex128)
        for c in range(nd):
            e[c] = 1.0
            m[:, c] = self.apply(e)
            e[c] = 0.0
        return m


def hf_energy_closed_form(n_qubits: int, n_electrons: int, h0, h, g) -> float:
    """<HF|H|HF> = h0 + sum_i h_ii + 1/2 sum_ij [(ii|jj) - delta_{s_i s_j} (ij|ji)]
    over occupied spin orbitals i, j (Slater-Condon rule for a single
    determinant)."""
    occ = range(n_electrons)
    e = h0 + sum(h[i // 2, i // 2] for i in occ)
    for i in occ:
        for j in occ:
            e += 0.5 * g[i // 2, i // 2, j // 2, j // 2]
            if i % 2 == j % 2:
                e -= 0.5 * g[i // 2, j // 2, j // 2, i // 2]
    return float(e)


def grad_at_hf_closed_form(n_electrons: int, excs, h, g) -> np.ndarray:
    """dE/dtheta_j at theta = 0 is 2 <HF|H T_j|HF>:
    singles (i -> a): 2 F_ia, F_ia = h_ia + sum_{k occ} [(ia|kk) - delta_{s_i s_k} (ik|ka)];
    doubles (i, j -> a, b): 2 [(ia|jb) d(s_i,s_a) d(s_j,s_b) - (ib|ja) d(s_i,s_b) d(s_j,s_a)]."""
    out = []
    for exc in excs:
        if len(exc) == 2:
            i, a = exc
            f = h[i // 2, a // 2]
            for k in range(n_electrons):
                f += g[i // 2, a // 2, k // 2, k // 2]
                if i % 2 == k % 2:
                    f -= g[i // 2, k // 2, k // 2, a // 2]
            out.append(2.0 * f)
        else:
            i, j, a, b = exc
            v = 0.0
            if i % 2 == a % 2 and j % 2 == b % 2:
                v += g[i // 2, a // 2, j // 2, b // 2]
            if i % 2 == b % 2 and j % 2 == a % 2:
                v -= g[i // 2, b // 2, j // 2, a // 2]
            out.append(2.0 * v)
    return np.array(out)


# --------------------------------------------------------------------------
# Energy, gradient, FCI, VQE
# --------------------------------------------------------------------------

class Problem:
    """One VQE instance: integrals + UCCSD on the HF reference."""

    def __init__(self, n_qubits: int, n_electrons: int, h0, h, g, excs=None):
        self.space = Space(n_qubits, n_electrons)
        self.ham = Hamiltonian(self.space, h0, h, g)
        self.excs = uccsd_excitations(n_qubits, n_electrons) if excs is None else list(excs)
        self.h0, self.h, self.g = h0, h, g

    @property
    def n_params(self) -> int:
        return len(self.excs)

    def state(self, theta) -> np.ndarray:
        return prepare(self.space, self.excs, theta)

    def energy(self, theta) -> float:
        return self.ham.expectation(self.state(theta))

    def grad_shift(self, theta, idx=None) -> np.ndarray:
        """Exact gradient by a four-term shift rule.

        T_j - T_j^dag has eigenvalues {0, +i, -i}, so E restricted to theta_j is
        a trigonometric polynomial with frequencies {1, 2}.  Matching
        d/dtheta on sin/cos of both frequencies gives
          dE = [E(+pi/4) - E(-pi/4)] - (sqrt2 - 1)/2 [E(+pi/2) - E(-pi/2)],
        with E(+-d) the energy at theta_j +- d (derived here; the same family
        of rules appears for excitation gates in the literature).
        """
        theta = np.asarray(theta, dtype=np.float64)
        idx = range(theta.size) if idx is None else idx
        c2 = (math.sqrt(2.0) - 1.0) / 2.0
        out = []
        for j in idx:
            def e(d):
                t = theta.copy()
                t[j] += d
                return self.energy(t)
            out.append((e(math.pi / 4) - e(-math.pi / 4)) - c2 * (e(math.pi / 2) - e(-math.pi / 2)))
        return np.array(out)

    def grad_fd(self, theta, h=1e-5, idx=None) -> np.ndarray:
        theta = np.asarray(theta, dtype=np.float64)
        idx = range(theta.size) if idx is None else idx
        out = []
        for j in idx:
            tp = theta.copy(); tp[j] += h
            tm = theta.copy(); tm[j] -= h
            out.append((self.energy(tp) - self.energy(tm)) / (2 * h))
        return np.array(out)

    def fci(self) -> float:
        """Lowest eigenvalue of H in the (N, S_z) sector."""
        nd = self.space.ndet
        if nd <= 2500:
            return float(scipy.linalg.eigvalsh(self.ham.matrix())[0])
        op = scipy.sparse.linalg.LinearOperator((nd, nd), matvec=self.ham.apply,
                                                dtype=np.complex128)
        w = scipy.sparse.linalg.eigsh(op, k=1, which="SA", tol=1e-12,
                                      v0=self.space.hf() + 1e-3)[0]
        return float(w[0])

    def vqe(self, theta0=None, gtol=1e-8, maxiter=200):
        """BFGS on E(theta) with exact (shift-rule) gradients (Sec. 3.1 names
        BFGS among the optimizers).  Returns scipy's OptimizeResult."""
        x0 = np.zeros(self.n_params) if theta0 is None else np.asarray(theta0, float)
        fun = lambda t: (self.energy(t), self.grad_shift(t))
        return scipy.optimize.minimize(fun, x0, jac=True, method="BFGS",
                                       options={"gtol": gtol, "maxiter": maxiter})


# --------------------------------------------------------------------------
# ADAPT-VQE (Sec. 2.1, "ADAPT-VQE algorithm"; Fig. 2(b))
# --------------------------------------------------------------------------

def _shift_rule(e):
    """d/dt of a frequency-{1, 2} trigonometric polynomial at 0 from its
    values e(+-pi/4), e(+-pi/2) (the four-term rule of Problem.grad_shift)."""
    c2 = (math.sqrt(2.0) - 1.0) / 2.0
    return (e(math.pi / 4) - e(-math.pi / 4)) - c2 * (e(math.pi / 2) - e(-math.pi / 2))


def pool_gradient(problem: Problem, theta, pool):
    """Energy of U(theta)|HF> and, for every pool operator A_k, the derivative
    of the energy with respect to the angle of exp(t A_k) applied after
    U(theta), at t = 0 (the quantity ADAPT-VQE ranks the pool by).

    Each derivative is taken from the energy of the extended state at four
    angles (exact for these generators), not from a commutator formula.
    """
    psi = problem.state(theta)
    ham = problem.ham
    e0 = ham.expectation(psi)
    out = []
    for op in pool:
        out.append(_shift_rule(
            lambda t: ham.expectation(apply_excitation(problem.space, psi, op, t))))
    return e0, np.array(out)


def adapt_select(grad, tie_tol):
    """Index of the pool operator to add: the lowest index whose |gradient|
    is within tie_tol of the largest (reading: ties, e.g. the alpha/beta
    partners of a spin-adapted Hamiltonian, go to the lower index)."""
    mag = np.abs(np.asarray(grad, dtype=np.float64))
    return int(np.nonzero(mag >= mag.max() - tie_tol)[0][0])


def adapt(n_qubits, n_electrons, h0, h, g, pool=None, grad_tol=1e-3, max_operators=None,
          tie_tol=1e-10, gtol=1e-8, maxiter=400, record=None):
    """ADAPT-VQE from the identity ansatz (the HF state).

    Each round: pool gradients at the current optimum; stop when their L2
    norm is below grad_tol (or max_operators are in); otherwise append the
    selected operator (applied last, angle 0, earlier angles kept) and run
    BFGS over all angles.  An operator may be selected more than once.
    Returns (selected indices, final angles, energies, gradient norms), the
    last two with one entry per ansatz size 0 .. len(selected).  If
    ``record`` is a list, (angles, pool gradient) of every step are appended.
    """
    if pool is None:
        pool = uccsd_excitations(n_qubits, n_electrons)
    pool = list(pool)
    cap = len(pool) if max_operators is None else int(max_operators)
    sel, theta = [], np.zeros(0)
    energies, norms = [], []
    while True:
        prob = Problem(n_qubits, n_electrons, h0, h, g, excs=[pool[i] for i in sel])
        e, gp = pool_gradient(prob, theta, pool)
        if record is not None:
            record.append((theta.copy(), gp))
        energies.append(e)
        norms.append(float(np.linalg.norm(gp)))
        if norms[-1] < grad_tol or len(sel) >= cap:
            break
        sel.append(adapt_select(gp, tie_tol))
        prob = Problem(n_qubits, n_electrons, h0, h, g, excs=[pool[i] for i in sel])
        theta = prob.vqe(theta0=np.append(theta, 0.0), gtol=gtol, maxiter=maxiter).x
    return sel, theta, np.array(energies), np.array(norms)


# --------------------------------------------------------------------------
# Trotter steps (Sec. 2.1, ansatz list: the depth of UCCSD)
# --------------------------------------------------------------------------

class TrotterProblem:
    """UCCSD (or any excitation list) with `steps` Trotter steps and shared
    angles.  The gradient is the chain rule over the expanded product: each
    angle appears `steps` times with weight 1/steps, and each appearance's
    derivative is exact (shift rule of the expanded problem)."""

    def __init__(self, n_qubits, n_electrons, h0, h, g, steps, excs=None):
        self.base = Problem(n_qubits, n_electrons, h0, h, g, excs=excs)
        self.steps = int(steps)
        self.excs = self.base.excs
        self.expanded = Problem(n_qubits, n_electrons, h0, h, g,
                                excs=trotter_expand(self.excs, np.zeros(len(self.excs)), steps)[0])

    @property
    def n_params(self):
        return len(self.excs)

    def state(self, theta):
        return self.expanded.state(trotter_expand(self.excs, theta, self.steps)[1])

    def energy(self, theta):
        return self.expanded.energy(trotter_expand(self.excs, theta, self.steps)[1])

    def grad(self, theta):
        g = self.expanded.grad_shift(trotter_expand(self.excs, theta, self.steps)[1])
        return g.reshape(self.steps, -1).sum(axis=0) / self.steps
