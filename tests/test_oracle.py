"""Pins of the CPU oracle against things other than itself: brute-force Fock
space matrices, closed forms, library routines (expm, eigh), invariants and a
textbook two-level case.  No GPU, no HIP library."""
import math

import numpy as np
import pytest

from oracle import brute as B
from oracle import fermion as F
from oracle import pauli as P
from vqe_inputs import random_integrals

SMALL = [(4, 2), (5, 2), (5, 3), (6, 3), (6, 2), (7, 4), (8, 4)]


def _problem(n, ne, seed=11):
    h0, h, g = random_integrals(n, seed)
    return F.Problem(n, ne, h0, h, g), (h0, h, g)


@pytest.mark.parametrize("n", [4, 5, 6])
def test_brute_hamiltonian_invariants(n):
    h0, h, g = random_integrals(n, 3)
    H = B.hamiltonian(n, h0, h, g)
    N, Sz = B.number_ops(n)
    assert np.abs(H - H.T).max() < 1e-13
    assert np.abs(H @ N - N @ H).max() < 1e-12
    assert np.abs(H @ Sz - Sz @ H).max() < 1e-12


@pytest.mark.parametrize("n,ne", SMALL)
def test_sigma_matches_brute_force(n, ne):
    prob, (h0, h, g) = _problem(n, ne)
    Hb = B.hamiltonian(n, h0, h, g)
    idx = prob.space.bits
    ref_idx = B.sector_indices(n, prob.space.na, prob.space.nb)
    assert sorted(idx.tolist()) == ref_idx.tolist()
    rng = np.random.default_rng(5)
    v = rng.normal(size=idx.size) + 1j * rng.normal(size=idx.size)
    assert np.abs(prob.ham.apply(v) - Hb[np.ix_(idx, idx)] @ v).max() < 1e-12


@pytest.mark.parametrize("n,ne", SMALL + [(12, 6), (16, 8)])
def test_energy_at_zero_is_closed_form_hf(n, ne):
    prob, (h0, h, g) = _problem(n, ne)
    e0 = prob.energy(np.zeros(prob.n_params))
    assert abs(e0 - F.hf_energy_closed_form(n, ne, h0, h, g)) < 1e-12
    if n <= 8:
        Hb = B.hamiltonian(n, h0, h, g)
        hf = (1 << ne) - 1
        assert abs(e0 - Hb[hf, hf]) < 1e-12


def test_uccsd_counts():
    # spin-conserving singles and doubles on the HF reference
    for n, m in [(4, 3), (12, 117), (16, 360), (20, 875), (24, 1818)]:
        excs = F.uccsd_excitations(n, n // 2)
        assert len(excs) == m
    # 4 qubits: two singles (one per spin) then the one alpha-beta double
    assert F.uccsd_excitations(4, 2) == [(0, 2), (1, 3), (0, 1, 2, 3)]


@pytest.mark.parametrize("n,ne", [(4, 2), (5, 3), (6, 3), (7, 3)])
def test_excitation_gate_matches_expm(n, ne):
    prob, _ = _problem(n, ne)
    rng = np.random.default_rng(1)
    for exc in prob.excs:
        theta = rng.uniform(-1.5, 1.5)
        psi = rng.normal(size=prob.space.ndet) + 1j * rng.normal(size=prob.space.ndet)
        got = F.apply_excitation(prob.space, psi, exc, theta)
        U = B.excitation_unitary(n, exc, theta)
        full = prob.space.to_statevector(psi)
        ref = U @ full
        assert np.abs(ref[prob.space.bits] - got).max() < 1e-12
        assert np.abs(np.delete(ref, prob.space.bits)).max() < 1e-12


@pytest.mark.parametrize("n", [4, 5, 6])
def test_pauli_jw_matches_brute_force(n):
    h0, h, g = random_integrals(n, 9)
    HP = P.jw_hamiltonian(n, 0.7, h, g)
    assert np.abs(P.matrix(HP, n) - B.hamiltonian(n, 0.7, h, g)).max() < 1e-12
    # real symmetric Hamiltonian: every folded coefficient is real
    P.folded_terms(HP)


@pytest.mark.parametrize("n,ne", [(4, 2), (5, 3), (6, 3)])
def test_rotation_products_match_expm(n, ne):
    rng = np.random.default_rng(2)
    for exc in F.uccsd_excitations(n, ne):
        rots = P.excitation_rotations(n, exc)
        assert len(rots) == (2 if len(exc) == 2 else 8)
        assert len({x for x, _, _ in rots}) == 1          # one shared x-mask
        assert all(abs(abs(s) - (1.0 if len(exc) == 2 else 0.25)) < 1e-15 for *_, s in rots)
        theta = rng.uniform(-1, 1)
        psi = rng.normal(size=1 << n) + 1j * rng.normal(size=1 << n)
        out = psi.copy()
        for x, z, s in rots:
            out = P.apply_rotation(out, n, (x, z), s * theta)
        assert np.abs(out - B.excitation_unitary(n, exc, theta) @ psi).max() < 1e-12


@pytest.mark.parametrize("n,ne", [(8, 4), (9, 4), (10, 5)])
def test_ci_energy_matches_dense_pauli(n, ne):
    prob, (h0, h, g) = _problem(n, ne, seed=21)
    HP = P.jw_hamiltonian(n, h0, h, g)
    theta = np.random.default_rng(3).uniform(-0.3, 0.3, prob.n_params)
    psi = P.prepare(n, ne, prob.excs, theta)
    # invariants of the dense evolution: norm, reality, particle number, sector
    assert abs(np.linalg.norm(psi) - 1) < 1e-13
    assert np.abs(psi.imag).max() < 1e-14
    outside = np.delete(psi, prob.space.bits)
    assert np.abs(outside).max() < 1e-14
    occ = np.array([bin(b).count("1") for b in range(1 << n)])
    assert abs(np.sum(np.abs(psi) ** 2 * occ) - ne) < 1e-12
    assert np.abs(psi[prob.space.bits] - prob.state(theta)).max() < 1e-12
    assert abs(P.energy(HP, psi, n) - prob.energy(theta)) < 1e-11


@pytest.mark.parametrize("n,ne", [(4, 2), (6, 3), (8, 4), (12, 6)])
def test_gradient_at_hf_closed_form(n, ne):
    prob, (h0, h, g) = _problem(n, ne)
    got = prob.grad_shift(np.zeros(prob.n_params))
    ref = F.grad_at_hf_closed_form(ne, prob.excs, h, g)
    assert np.abs(got - ref).max() < 1e-12
    assert np.abs(ref).max() > 1e-2  # random integrals are not SCF: nonzero


@pytest.mark.parametrize("n,ne", [(5, 2), (6, 3), (8, 4)])
def test_shift_rule_vs_central_difference(n, ne):
    prob, _ = _problem(n, ne)
    theta = np.random.default_rng(4).uniform(-0.5, 0.5, prob.n_params)
    assert np.abs(prob.grad_shift(theta) - prob.grad_fd(theta, h=1e-5)).max() < 1e-8


@pytest.mark.parametrize("n,ne", SMALL)
def test_fci_matches_brute_force_sector(n, ne):
    prob, (h0, h, g) = _problem(n, ne)
    Hb = B.hamiltonian(n, h0, h, g)
    idx = B.sector_indices(n, prob.space.na, prob.space.nb)
    ref = np.linalg.eigvalsh(Hb[np.ix_(idx, idx)])[0]
    assert abs(prob.fci() - ref) < 1e-11


def test_fci_lanczos_branch_one_body_closed_form():
    """Above 2,500 determinants the sector FCI switches from dense eigh to
    Lanczos (eigsh) on the sigma-vector.  With the two-body integrals zero
    the ground energy has a closed form: the alpha and the beta electrons
    fill the lowest eigenvalues of h (spin-adapted spatial orbitals).  16
    qubits, 6 electrons: 3,136 determinants."""
    n, ne = 16, 6
    _, h, g = random_integrals(n, 1616)
    prob = F.Problem(n, ne, 0.0, h, np.zeros_like(g))
    assert prob.space.ndet > 2500
    eps = np.linalg.eigvalsh(h)
    na, nb = (ne + 1) // 2, ne // 2
    assert abs(prob.fci() - (eps[:na].sum() + eps[:nb].sum())) < 1e-10


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_vqe_4q_reaches_fci(seed):
    h0, h, g = random_integrals(4, seed)
    prob = F.Problem(4, 2, h0, h, g)
    res = prob.vqe(maxiter=50)
    assert abs(res.fun - prob.fci()) < 1e-9


def test_vqe_6q_variational_bound():
    prob, _ = _problem(6, 3, seed=2)
    res = prob.vqe(maxiter=200)
    assert res.fun >= prob.fci() - 1e-10
    assert res.fun < prob.energy(np.zeros(prob.n_params))


def test_two_level_closed_form():
    """H2-like 4-qubit model (bonding 0 / antibonding 1 orbitals): with h_01 = 0
    and every (pq|rs) with an odd number of 1-indices zero, the HF determinant
    couples only to the doubly excited one, so min_theta E(theta) over the
    double alone is the 2x2 ground state
      E = (E1 + E2)/2 - sqrt((E1 - E2)^2 / 4 + K^2),
    E1 = 2 h00 + (00|00), E2 = 2 h11 + (11|11), K = (01|01)."""
    h = np.diag([-1.25, -0.47])
    g = np.zeros((2, 2, 2, 2))
    vals = {(0, 0, 0, 0): 0.67, (1, 1, 1, 1): 0.70, (0, 0, 1, 1): 0.66, (0, 1, 0, 1): 0.18}
    for (p, q, r, s), v in vals.items():
        for a, b, c, d in ((p, q, r, s), (q, p, r, s), (p, q, s, r), (q, p, s, r),
                           (r, s, p, q), (s, r, p, q), (r, s, q, p), (s, r, q, p)):
            g[a, b, c, d] = v
    prob = F.Problem(4, 2, 0.0, h, g, excs=[(0, 1, 2, 3)])
    E1 = 2 * h[0, 0] + g[0, 0, 0, 0]
    E2 = 2 * h[1, 1] + g[1, 1, 1, 1]
    K = g[0, 1, 0, 1]
    ref = 0.5 * (E1 + E2) - math.sqrt(0.25 * (E1 - E2) ** 2 + K * K)
    thetas = np.linspace(-math.pi / 2, math.pi / 2, 2001)
    es = [prob.energy([t]) for t in thetas]
    t0 = thetas[int(np.argmin(es))]
    import scipy.optimize
    r = scipy.optimize.minimize_scalar(lambda t: prob.energy([t]), bracket=(t0 - 0.01, t0 + 0.01))
    assert abs(r.fun - ref) < 1e-12
    assert abs(prob.fci() - ref) < 1e-12
    # the symmetric model has 15 Pauli terms (the H2 count), generic 4q has 27
    assert len(P.jw_hamiltonian(4, 0.0, h, g)) == 15
    assert len(P.jw_hamiltonian(4, *random_integrals(4, 1))) == 27


def test_term_and_group_counts_12q():
    terms = P.folded_terms(P.jw_hamiltonian(12, *random_integrals(12, 2)))
    xs = {x for x, _ in terms}
    diag = [k for k in terms if k[0] == 0]
    assert (len(terms), len(xs), len(diag)) == (1819, 286, 79)


# ----------------------------------------------------------------- MLP oracle
from oracle import mlp as NN  # noqa: E402


def test_bf16_rounding_known_values():
    # 1 + 2^-8 is halfway between bf16 neighbours 1 and 1 + 2^-7: ties to even -> 1
    assert NN.bf16(1.0 + 2.0 ** -8) == 1.0
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 and 1 + 2^-6: ties to even -> 1 + 2^-6
    assert NN.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6
    assert NN.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7   # above the tie
    assert NN.bf16(-3.14159265) == -3.140625
    assert NN.bf16(65504.0) == 65536.0
    assert np.isnan(NN.bf16(np.nan))
    x = np.random.default_rng(0).normal(size=1000).astype(np.float32).astype(np.float64)
    rel = np.abs(NN.bf16(x) - x) / np.abs(x)
    assert rel.max() <= 2.0 ** -8 + 1e-12


def test_gelu_closed_forms():
    assert NN.gelu(0.0) == 0.0
    assert abs(NN.gelu(1.0) - 0.8413447460685429) < 1e-15      # Phi(1)
    z = np.linspace(-4, 4, 41)
    h = 1e-6
    fd = (NN.gelu(z + h) - NN.gelu(z - h)) / (2 * h)
    assert np.abs(fd - NN.gelu_grad(z)).max() < 1e-8


def test_mlp_gradient_vs_central_differences():
    widths = [5, 7, 6, 4]
    rng = np.random.default_rng(3)
    p = NN.init_params(widths, 1) + rng.normal(0, 0.1, NN.n_params(widths))
    x = rng.normal(size=(9, 5))
    y = rng.normal(size=(9, 4))
    _, g = NN.loss_and_grad(p, widths, x, y, rounding=False)
    fd = np.empty_like(p)
    for k in range(p.size):
        e = np.zeros_like(p)
        e[k] = 1e-6
        fd[k] = (NN.loss_and_grad(p + e, widths, x, y, False)[0] -
                 NN.loss_and_grad(p - e, widths, x, y, False)[0]) / 2e-6
    assert np.abs(fd - g).max() < 1e-8
    assert NN.n_params([37, 256, 256, 360]) == 168040


def test_adam_first_step_closed_form():
    # t = 1: m_hat = g, v_hat = g^2, so the step is lr * g / (|g| + eps)
    p = np.array([0.5, -1.0, 2.0])
    g = np.array([0.1, -3.0, 0.0])
    p1, m, v = NN.adam_step(p, g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=1e-8)
    assert np.allclose(p1, p - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)


# ---------------------------------------------------------------- ADAPT-VQE

@pytest.mark.parametrize("n,ne", [(4, 2), (6, 3), (8, 4)])
def test_pool_gradient_at_identity_is_hf_closed_form(n, ne):
    h0, h, g = random_integrals(n, 11)
    pool = F.uccsd_excitations(n, ne)
    e, got = F.pool_gradient(F.Problem(n, ne, h0, h, g, excs=[]), np.zeros(0), pool)
    assert abs(e - F.hf_energy_closed_form(n, ne, h0, h, g)) < 1e-12
    assert np.abs(got - F.grad_at_hf_closed_form(ne, pool, h, g)).max() < 1e-12


@pytest.mark.parametrize("n,ne", [(5, 2), (6, 3)])
def test_pool_gradient_matches_fock_space_commutator(n, ne):
    """d/dt <psi|e^{-tG} H e^{tG}|psi> at 0 = <psi|[H, G]|psi> = 2 Re <H psi|G psi>,
    with G = T - T^dag built from the occupation-number ladder matrices."""
    h0, h, g = random_integrals(n, 5)
    pool = F.uccsd_excitations(n, ne)
    rng = np.random.default_rng(9)
    sel = [int(k) for k in rng.integers(0, len(pool), 4)]
    prob = F.Problem(n, ne, h0, h, g, excs=[pool[k] for k in sel])
    theta = rng.uniform(-0.6, 0.6, len(sel))
    e, got = F.pool_gradient(prob, theta, pool)
    psi = prob.space.to_statevector(prob.state(theta))
    Hb = B.hamiltonian(n, h0, h, g)
    hpsi = Hb @ psi
    ref = [2.0 * np.real(np.vdot(hpsi, B.excitation_generator(n, op) @ psi)) for op in pool]
    assert abs(e - np.real(np.vdot(psi, hpsi))) < 1e-11
    assert np.abs(got - np.array(ref)).max() < 1e-11


def test_pool_gradient_of_a_repeated_operator_vanishes_at_optimum():
    """Appending the last operator again adds to its angle: at a stationary
    point of E in that angle the pool gradient of the operator is zero."""
    h0, h, g = random_integrals(6, 3)
    pool = F.uccsd_excitations(6, 3)
    prob = F.Problem(6, 3, h0, h, g, excs=[pool[4]])
    th = prob.vqe(theta0=np.zeros(1), gtol=1e-12).x
    _, gp = F.pool_gradient(prob, th, pool)
    assert abs(gp[4]) < 1e-9
    assert np.abs(gp).max() > 1e-3


def test_adapt_select_tie_rule():
    assert F.adapt_select([0.1, -0.3, 0.3, 0.2], 1e-10) == 1
    assert F.adapt_select([0.1, -0.3, 0.3 + 1e-12, 0.2], 1e-10) == 1
    assert F.adapt_select([0.1, -0.3, 0.3 + 1e-6, 0.2], 1e-10) == 2
    assert F.adapt_select([0.0, 0.0], 1e-10) == 0


@pytest.mark.parametrize("seed", [1, 2])
def test_adapt_4q_reaches_fci(seed):
    h0, h, g = random_integrals(4, seed)
    sel, theta, es, norms = F.adapt(4, 2, h0, h, g, grad_tol=1e-6)
    fci = F.Problem(4, 2, h0, h, g).fci()
    assert abs(es[-1] - fci) < 1e-9
    assert norms[-1] < 1e-6
    assert len(sel) == len(theta) == len(es) - 1


def test_adapt_invariants_6q():
    """Energies never rise (each ansatz contains the previous one at its
    optimum), stay above the sector FCI, start at the HF energy, and the first
    operator is the closed-form HF gradient's pick."""
    h0, h, g = random_integrals(6, 4)
    pool = F.uccsd_excitations(6, 4)
    sel, theta, es, norms = F.adapt(6, 4, h0, h, g, grad_tol=1e-5)
    fci = F.Problem(6, 4, h0, h, g).fci()
    assert abs(es[0] - F.hf_energy_closed_form(6, 4, h0, h, g)) < 1e-12
    assert np.all(np.diff(es) <= 1e-12)
    assert es.min() >= fci - 1e-10
    assert abs(es[-1] - fci) < 1e-7
    assert sel[0] == F.adapt_select(F.grad_at_hf_closed_form(4, pool, h, g), 1e-10)


# ------------------------------------------------ pUCCD (hard-core bosons)

from oracle import hcb as HB  # noqa: E402


def _seniority_zero(space: F.Space, n_orb):
    """Indices of the determinants with every spatial orbital doubly occupied or
    empty, and the pair pattern of each."""
    idx, pats = [], []
    for k, b in enumerate(space.bits):
        b = int(b)
        pat = 0
        ok = True
        for p in range(n_orb):
            a_, b_ = (b >> (2 * p)) & 1, (b >> (2 * p + 1)) & 1
            if a_ != b_:
                ok = False
                break
            pat |= a_ << p
        if ok:
            idx.append(k)
            pats.append(pat)
    return np.array(idx), pats


@pytest.mark.parametrize("n_orb,n_pairs", [(2, 1), (3, 1), (4, 2), (5, 2), (6, 3)])
def test_hcb_matrix_is_projected_fermion_hamiltonian(n_orb, n_pairs):
    """The pair Hamiltonian equals the fermionic sector Hamiltonian restricted
    to seniority-zero determinants (entry by entry, signs included)."""
    h0, h, g = random_integrals(2 * n_orb, 17 + n_orb)
    fs = F.Space(2 * n_orb, 2 * n_pairs)
    Hf = F.Hamiltonian(fs, h0, h, g).matrix()
    idx, pats = _seniority_zero(fs, n_orb)
    sp = HB.Space(n_orb, n_pairs)
    assert len(idx) == sp.ndet
    order = [sp.index[p] for p in pats]
    Hb = HB.hamiltonian_matrix(sp, h0, h, g)
    assert np.abs(Hf[np.ix_(idx, idx)].real - Hb[np.ix_(order, order)]).max() < 1e-12
    assert np.abs(Hf[np.ix_(idx, idx)].imag).max() < 1e-14


@pytest.mark.parametrize("n_orb,n_pairs", [(3, 1), (4, 2), (5, 2)])
def test_puccd_energy_matches_fermion_pair_doubles(n_orb, n_pairs):
    """pUCCD on the pair space = the fermionic ansatz of the same pair double
    excitations (2i, 2i+1 -> 2a, 2a+1) applied to HF, at the same angles."""
    h0, h, g = random_integrals(2 * n_orb, 23 + n_orb)
    prob = HB.Problem(n_orb, n_pairs, h0, h, g)
    excs = [(2 * i, 2 * i + 1, 2 * a, 2 * a + 1) for i, a in prob.excs]
    fprob = F.Problem(2 * n_orb, 2 * n_pairs, h0, h, g, excs=excs)
    theta = np.random.default_rng(n_orb).uniform(-0.8, 0.8, prob.n_params)
    assert abs(prob.energy(theta) - fprob.energy(theta)) < 1e-12
    assert abs(prob.energy(np.zeros(prob.n_params)) -
               F.hf_energy_closed_form(2 * n_orb, 2 * n_pairs, h0, h, g)) < 1e-12
    assert np.abs(prob.grad_shift(theta) - fprob.grad_fd(theta, h=1e-5)).max() < 1e-8


def test_puccd_counts_ch3f():
    """11 active orbitals with 7 pairs: 28 parameters, 11 qubits."""
    assert len(HB.puccd_excitations(11, 7)) == 28
    assert HB.Space(11, 7).ndet == 330


def test_hcb_ground_state_above_fermion_fci():
    """The pair space is a subspace of the sector: its lowest energy is an
    upper bound to the sector FCI; the pUCCD optimum lies above both."""
    import scipy.optimize
    n_orb, n_pairs = 4, 2
    h0, h, g = random_integrals(8, 5)
    prob = HB.Problem(n_orb, n_pairs, h0, h, g)
    fci = F.Problem(8, 4, h0, h, g).fci()
    e0 = prob.ground()
    assert e0 >= fci - 1e-12
    res = scipy.optimize.minimize(lambda t: (prob.energy(t), prob.grad_shift(t)),
                                  np.zeros(prob.n_params), jac=True, method="BFGS")
    assert res.fun >= e0 - 1e-10
    assert res.fun < prob.energy(np.zeros(prob.n_params))


# ------------------------------------------- Trotter steps, k-UpCCGSD

def _sector_generator(space, exc):
    """T - T^dag on the sector, from the brute-force Fock matrices."""
    G = B.excitation_generator(space.n, exc)
    return G[np.ix_(space.bits, space.bits)]


@pytest.mark.parametrize("n,ne", [(4, 2), (6, 3)])
def test_trotter_converges_to_the_unfactorised_exponential(n, ne):
    """U_steps -> exp(sum_j theta_j (T_j - T_j^dag)) as steps grows (first-order
    Trotter: error ~ 1/steps); steps = 1 is plain UCCSD."""
    import scipy.linalg
    h0, h, g = random_integrals(n, 31)
    excs = F.uccsd_excitations(n, ne)
    theta = np.random.default_rng(3).uniform(-0.5, 0.5, len(excs))
    space = F.Space(n, ne)
    K = sum(t * _sector_generator(space, e) for t, e in zip(theta, excs))
    exact = scipy.linalg.expm(K) @ space.hf()
    errs = []
    for steps in (1, 2, 8, 64):
        tp = F.TrotterProblem(n, ne, h0, h, g, steps)
        errs.append(np.linalg.norm(tp.state(theta) - exact))
    assert np.linalg.norm(F.TrotterProblem(n, ne, h0, h, g, 1).state(theta) -
                          F.Problem(n, ne, h0, h, g).state(theta)) < 1e-14
    assert errs[0] > errs[1] > errs[2] > errs[3]
    assert errs[3] < errs[0] / 20


@pytest.mark.parametrize("n,ne,steps", [(4, 2, 2), (5, 2, 3), (6, 3, 2)])
def test_trotter_gradient_vs_central_difference(n, ne, steps):
    h0, h, g = random_integrals(n, 41)
    tp = F.TrotterProblem(n, ne, h0, h, g, steps)
    theta = np.random.default_rng(7).uniform(-0.5, 0.5, tp.n_params)
    fd = []
    for j in range(tp.n_params):
        a, b = theta.copy(), theta.copy()
        a[j] += 1e-5
        b[j] -= 1e-5
        fd.append((tp.energy(a) - tp.energy(b)) / 2e-5)
    assert np.abs(tp.grad(theta) - np.array(fd)).max() < 1e-8


def test_kupccgsd_layer_counts_and_generators():
    """Counts: 2 C(n/2, 2) singles (even n) + C(n/2, 2) pair doubles; every
    gate equals expm(theta (T - T^dag)) on the sector, including singles that
    annihilate empty orbitals of the reference and pair moves between
    virtual orbitals."""
    import scipy.linalg
    assert len(F.kupccgsd_layer(4)) == 2 + 1
    assert len(F.kupccgsd_layer(8)) == 2 * 6 + 6
    assert len(F.kupccgsd_layer(7)) == 6 + 3 + 3   # 4 alpha, 3 beta orbitals; 3 pairs
    n, ne = 6, 2
    space = F.Space(n, ne)
    psi = np.random.default_rng(1).normal(size=space.ndet) + 0j
    psi /= np.linalg.norm(psi)
    for exc in F.kupccgsd_layer(n):
        ref = scipy.linalg.expm(0.37 * _sector_generator(space, exc)) @ psi
        assert np.abs(F.apply_excitation(space, psi, exc, 0.37) - ref).max() < 1e-12


def test_kupccgsd_vqe_bounds():
    """E(0) = E_HF; a 2-layer optimum lies between FCI and E_HF and below the
    1-layer optimum (the 2-layer ansatz contains the 1-layer one)."""
    n, ne = 4, 2
    h0, h, g = random_integrals(n, 9)
    fci = F.Problem(n, ne, h0, h, g).fci()
    res = []
    for k in (1, 2):
        prob = F.Problem(n, ne, h0, h, g, excs=F.kupccgsd_excitations(n, k))
        assert abs(prob.energy(np.zeros(prob.n_params)) -
                   F.hf_energy_closed_form(n, ne, h0, h, g)) < 1e-12
        th0 = np.random.default_rng(2).uniform(-0.1, 0.1, prob.n_params)
        res.append(prob.vqe(theta0=th0, gtol=1e-9).fun)
    assert res[1] >= fci - 1e-10
    assert res[1] <= res[0] + 1e-9


# ------------------------------------------------------- Bravyi-Kitaev

def _bk_permutation(n):
    """Pi |occupation bits> = |BK register>, from the Fenwick rows written out."""
    dim = 1 << n
    Pi = np.zeros((dim, dim))
    for occ in range(dim):
        b = 0
        for j in range(n):
            lo = j + 1 - ((j + 1) & -(j + 1))
            b |= (sum((occ >> k) & 1 for k in range(lo, j + 1)) & 1) << j
        Pi[b, occ] = 1.0
    return Pi


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 8])
def test_bk_ladder_is_permuted_fock_ladder(n):
    """The BK ladder operators equal the occupation-number ladder matrices in
    the encoded basis (Pi a Pi^T), for every orbital; the encoding is a
    permutation of the basis."""
    cr, an = B.ladder(n)
    Pi = _bk_permutation(n)
    assert np.array_equal(Pi @ Pi.T, np.eye(1 << n))
    for j in range(n):
        got_c = P.matrix(P.bk_ladder(n, j, True), n)
        got_a = P.matrix(P.bk_ladder(n, j, False), n)
        assert np.abs(got_c - Pi @ cr[j].toarray() @ Pi.T).max() < 1e-14
        assert np.abs(got_a - Pi @ an[j].toarray() @ Pi.T).max() < 1e-14
    for occ in range(1 << n):
        assert Pi[P.bk_encode(n, occ), occ] == 1.0


@pytest.mark.parametrize("n,ne", [(4, 2), (5, 2), (6, 3)])
def test_bk_hamiltonian_and_uccsd_match_jw(n, ne):
    """Same spectrum (the mapping only relabels the basis), and the BK UCCSD
    state is the permuted JW state with the same energy."""
    h0, h, g = random_integrals(n, 51 + n)
    Hj = P.matrix(P.jw_hamiltonian(n, h0, h, g), n)
    Hb = P.matrix(P.jw_hamiltonian(n, h0, h, g, mapping="bk"), n)
    assert np.abs(np.linalg.eigvalsh(Hj) - np.linalg.eigvalsh(Hb)).max() < 1e-11
    Pi = _bk_permutation(n)
    assert np.abs(Hb - Pi @ Hj @ Pi.T).max() < 1e-12
    excs = F.uccsd_excitations(n, ne)
    theta = np.random.default_rng(n).uniform(-0.5, 0.5, len(excs))
    pj = P.prepare(n, ne, excs, theta)
    pb = P.prepare(n, ne, excs, theta, mapping="bk")
    assert np.abs(pb - Pi @ pj).max() < 1e-12
    prob = F.Problem(n, ne, h0, h, g)
    assert abs(np.real(np.vdot(pb, Hb @ pb)) - prob.energy(theta)) < 1e-11
