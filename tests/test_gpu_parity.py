"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.  Tolerances: energies and gradients 1e-10 Ha absolute
(FP64 throughout; the only differences are summation order and FMA
contraction, ~1e-14 here); amplitudes 1e-12."""
import math

import numpy as np
import pytest

import paper_2311_01242_amd as vq
from oracle import fermion as F
from oracle import pauli as P
from vqe_inputs import random_integrals, scan_integrals, uniform_theta

pytestmark = pytest.mark.gpu

TOL_E = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield


def _pair(n, ne, seed):
    h0, h, g = random_integrals(n, seed)
    return (vq.Hamiltonian.from_integrals(n, h0, h, g), vq.Ansatz.uccsd(n, ne),
            F.Problem(n, ne, h0, h, g))


def _new_state(n):
    """Statevector borrowed from a torch complex128 tensor (the wrap path)."""
    import torch
    t = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    return vq.State.wrap(t), t


def _read(t):
    import torch
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("n,ne", [(4, 2), (5, 2), (6, 3), (7, 4), (8, 4), (12, 6), (13, 6)])
def test_energy_at_theta_zero_is_hf(n, ne):
    H, A, prob = _pair(n, ne, 100 + n)
    e, g = vq.energy_grad(H, A, ne, np.zeros(A.n_params))
    assert abs(e - F.hf_energy_closed_form(n, ne, prob.h0, prob.h, prob.g)) < TOL_E
    assert np.abs(g - F.grad_at_hf_closed_form(ne, prob.excs, prob.h, prob.g)).max() < TOL_E


@pytest.mark.parametrize("n,ne", [(4, 2), (5, 3), (6, 3), (8, 4), (9, 4), (10, 5)])
def test_energy_and_gradient_vs_oracle(n, ne):
    H, A, prob = _pair(n, ne, 200 + n)
    theta = uniform_theta(300 + n, A.n_params, -0.4, 0.4)
    e, g = vq.energy_grad(H, A, ne, theta)
    assert abs(e - prob.energy(theta)) < TOL_E
    assert np.abs(g - prob.grad_shift(theta)).max() < TOL_E
    e2, none = vq.energy_grad(H, A, ne, theta, grad=False)
    assert none is None and abs(e2 - e) < 1e-14


def test_gradient_12q_sampled_components_and_fd():
    h0, h, g = scan_integrals(12, 2)(1.3)
    H = vq.Hamiltonian.from_integrals(12, h0, h, g)
    A = vq.Ansatz.uccsd(12, 6)
    prob = F.Problem(12, 6, h0, h, g)
    theta = uniform_theta(7, A.n_params)
    e, grad = vq.energy_grad(H, A, 6, theta)
    assert abs(e - prob.energy(theta)) < TOL_E
    idx = sorted(np.random.default_rng(1).choice(A.n_params, 24, replace=False).tolist())
    assert np.abs(grad[idx] - prob.grad_shift(theta, idx)).max() < TOL_E
    # adjoint vs central finite differences of the GPU energy, h = 1e-5
    fd = []
    for j in idx[:8]:
        tp, tm = theta.copy(), theta.copy()
        tp[j] += 1e-5
        tm[j] -= 1e-5
        fd.append((vq.energy_grad(H, A, 6, tp, grad=False)[0] -
                   vq.energy_grad(H, A, 6, tm, grad=False)[0]) / 2e-5)
    assert np.abs(grad[idx[:8]] - np.array(fd)).max() < 1e-6


def test_bitwise_reproducible():
    H, A, _ = _pair(10, 5, 3)
    theta = uniform_theta(3, A.n_params)
    r1 = vq.energy_grad(H, A, 5, theta)
    r2 = vq.energy_grad(H, A, 5, theta)
    assert r1[0] == r2[0] and np.array_equal(r1[1], r2[1])


@pytest.mark.parametrize("n,ne", [(6, 3), (9, 4)])
def test_statevector_matches_oracle(n, ne):
    H, A, prob = _pair(n, ne, 400 + n)
    theta = uniform_theta(5, A.n_params, -0.5, 0.5)
    st, t = _new_state(n)
    st.prepare_hf(ne)
    st.apply_ansatz(A, theta)
    arr = _read(t)
    ref = prob.space.to_statevector(prob.state(theta))
    assert np.abs(arr - ref).max() < 1e-12
    assert abs(st.expectation(H) - prob.energy(theta)) < TOL_E


def test_rotation_ansatz_matches_excitation_ansatz():
    n, ne = 6, 3
    H, A, prob = _pair(n, ne, 17)
    xs, zs, ps, ss = [], [], [], []
    for p, exc in enumerate(prob.excs):
        for x, z, s in P.excitation_rotations(n, exc):
            xs.append(x); zs.append(z); ps.append(p); ss.append(s)
    R = vq.Ansatz.from_rotations(n, len(prob.excs), xs, zs, ps, ss)
    theta = uniform_theta(9, A.n_params, -0.5, 0.5)
    e1, g1 = vq.energy_grad(H, A, ne, theta)
    e2, g2 = vq.energy_grad(H, R, ne, theta)
    assert abs(e1 - e2) < TOL_E and np.abs(g1 - g2).max() < TOL_E
    assert abs(e2 - prob.energy(theta)) < TOL_E
    st, t = _new_state(n)
    st.prepare_hf(ne)
    st.apply_ansatz(R, theta)
    arr = _read(t)
    assert np.abs(arr - P.prepare(n, ne, prob.excs, theta)).max() < 1e-12


def test_general_pauli_rotations_and_expectation():
    """Complex states: arbitrary Pauli rotations (incl. diagonal ones and odd
    numbers of Y) against the dense-Pauli oracle, then <psi|H|psi>."""
    n = 7
    h0, h, g = random_integrals(n, 23)
    H = vq.Hamiltonian.from_integrals(n, h0, h, g)
    HP = P.jw_hamiltonian(n, h0, h, g)
    rng = np.random.default_rng(8)
    st, t = _new_state(n)
    st.prepare_hf(3)
    ref = np.zeros(1 << n, np.complex128)
    ref[7] = 1.0
    rots = [(0, 0b101, 0.3), (0b11, 0b10, 0.7), (0b1000001, 0b1000000, -1.1), (0b110, 0b110, 0.4)]
    rots += [(int(rng.integers(0, 1 << n)), int(rng.integers(0, 1 << n)), float(rng.uniform(-2, 2)))
             for _ in range(12)]
    for x, z, ang in rots:
        st.apply_pauli_rotation(x, z, ang)
        ref = P.apply_rotation(ref, n, (x, z), ang)
    arr = _read(t)
    assert np.abs(arr - ref).max() < 1e-12
    assert np.abs(ref.imag).max() > 1e-3        # genuinely complex
    assert abs(st.expectation(H) - P.energy(HP, ref, n)) < TOL_E


def test_general_rotation_gradient_vs_fd():
    n, ne = 5, 2
    h0, h, g = random_integrals(n, 31)
    H = vq.Hamiltonian.from_integrals(n, h0, h, g)
    rng = np.random.default_rng(2)
    k = 10
    xs = rng.integers(0, 1 << n, k); zs = rng.integers(0, 1 << n, k)
    ps = rng.integers(0, 4, k); ss = rng.uniform(-1.5, 1.5, k)
    R = vq.Ansatz.from_rotations(n, 4, xs, zs, ps, ss)
    theta = rng.uniform(-1, 1, 4)
    e, grad = vq.energy_grad(H, R, ne, theta)
    HP = P.jw_hamiltonian(n, h0, h, g)

    def e_or(t):
        psi = np.zeros(1 << n, np.complex128)
        psi[(1 << ne) - 1] = 1
        for x, z, p, s in zip(xs, zs, ps, ss):
            psi = P.apply_rotation(psi, n, (int(x), int(z)), s * t[p])
        return P.energy(HP, psi, n)
    assert abs(e - e_or(theta)) < TOL_E
    # central differences of the oracle energy (h = 1e-5)
    shift = np.zeros(4)
    for j in range(4):
        tp, tm = theta.copy(), theta.copy()
        tp[j] += 1e-5; tm[j] -= 1e-5
        shift[j] = (e_or(tp) - e_or(tm)) / 2e-5
    assert np.abs(grad - shift).max() < 1e-7


def test_vqe_run_4q_reaches_fci():
    h0, h, g = random_integrals(4, 1)
    H = vq.Hamiltonian.from_integrals(4, h0, h, g)
    A = vq.Ansatz.uccsd(4, 2)
    theta, res, trace = vq.run_vqe(H, A, 2, max_iter=50, gtol=1e-8)
    prob = F.Problem(4, 2, h0, h, g)
    assert res.converged == 1
    assert abs(res.energy - prob.fci()) < 1e-9
    assert abs(trace[0] - F.hf_energy_closed_form(4, 2, h0, h, g)) < TOL_E
    assert abs(prob.energy(theta) - res.energy) < TOL_E


def test_batch_matches_single_state_path():
    specs = [(4, 2, 1), (6, 3, 2), (6, 3, 3), (7, 3, 4), (8, 4, 5), (6, 3, 6), (9, 4, 7),
             (13, 6, 8), (12, 6, 9), (15, 7, 10)]
    Hs, As, probs, thetas = [], [], [], []
    for n, ne, s in specs:
        H, A, prob = _pair(n, ne, 500 + s)
        Hs.append(H); As.append(A); probs.append(prob)
        thetas.append(uniform_theta(600 + s, A.n_params))
    b = vq.Batch(Hs, As, [ne for _, ne, _ in specs])
    flat = np.concatenate(thetas)
    e, g = b.energy_grad(flat)
    e2, g2 = b.energy_grad(flat)
    assert np.array_equal(e, e2) and np.array_equal(g, g2)     # graph replays are bitwise stable
    for i, (n, ne, _) in enumerate(specs):
        es, gs = vq.energy_grad(Hs[i], As[i], ne, thetas[i])
        gi = g[b.offsets[i]:b.offsets[i + 1]]
        # same kernels; batch and single-state launches may pick different
        # tilings (so different summation orders), hence 1e-12 not bitwise
        assert abs(e[i] - es) < 1e-12 and np.abs(gi - gs).max() < 1e-12
        assert abs(e[i] - probs[i].energy(thetas[i])) < TOL_E
    # a different theta replays through the same graph
    e3, _ = b.energy_grad(flat * 0.5)
    for i in range(len(specs)):
        assert abs(e3[i] - probs[i].energy(thetas[i] * 0.5)) < TOL_E


def test_torch_autograd_function():
    import torch
    H, A, prob = _pair(6, 3, 41)
    th = torch.tensor(uniform_theta(2, A.n_params), dtype=torch.float64, requires_grad=True)
    E = vq.EnergyGrad.apply(th, H, A, 3)
    (2.0 * E).backward()
    assert abs(E.item() - prob.energy(th.detach().numpy())) < TOL_E
    assert np.abs(th.grad.numpy() - 2.0 * prob.grad_shift(th.detach().numpy())).max() < TOL_E


@pytest.mark.parametrize("n,ne", [(14, 7), (15, 7), (16, 8)])
def test_sector_path_at_larger_sizes(n, ne):
    H, A, prob = _pair(n, ne, 700 + n)
    theta = uniform_theta(800 + n, A.n_params)
    e, g = vq.energy_grad(H, A, ne, theta)
    assert abs(e - prob.energy(theta)) < TOL_E
    idx = sorted(np.random.default_rng(n).choice(A.n_params, 6, replace=False).tolist())
    assert np.abs(g[idx] - prob.grad_shift(theta, idx)).max() < TOL_E


@pytest.mark.parametrize("fwd,adj,L", [(4096, 8192, 4), (8192, 16384, 6), (16384, 4096, 9),
                                       (65536, 131072, 12)])
def test_tiling_choices_agree(fwd, adj, L):
    """Small LDS budgets split runs into sub-runs with non-contiguous inner
    bits; every tiling must give the same energy and gradient."""
    n, ne = 12, 6
    H, A, prob = _pair(n, ne, 901)
    theta = uniform_theta(902, A.n_params)
    ref_e = prob.energy(theta)
    lib = vq.lib()
    try:
        assert lib.vqe_set_tuning(n, 0, fwd, adj, L) == 0
        A2 = vq.Ansatz.uccsd(n, ne)          # fresh handle: plans are made on first use
        e, g = vq.energy_grad(H, A2, ne, theta)
    finally:
        lib.vqe_set_tuning(n, 0, 0, 0, 0)
    e0, g0 = vq.energy_grad(H, A, ne, theta)
    assert abs(e - ref_e) < TOL_E
    assert abs(e - e0) < 1e-12 and np.abs(g - g0).max() < 1e-12


def test_workspace_switches_between_dense_and_sector_paths():
    """A rotation ansatz (dense H-apply, lambda written everywhere) followed by
    the UCCSD sector path on the same stream workspace."""
    n, ne = 8, 4
    H, A, prob = _pair(n, ne, 77)
    xs, zs, ps, ss = [], [], [], []
    for p, exc in enumerate(prob.excs):
        for x, z, s in P.excitation_rotations(n, exc):
            xs.append(x); zs.append(z); ps.append(p); ss.append(s)
    xs.append(1); zs.append(0); ps.append(0); ss.append(0.3)     # leaves the sector
    R = vq.Ansatz.from_rotations(n, len(prob.excs), xs, zs, ps, ss)
    theta = uniform_theta(78, A.n_params)
    vq.energy_grad(H, R, ne, theta)
    e, g = vq.energy_grad(H, A, ne, theta)
    assert abs(e - prob.energy(theta)) < TOL_E
    assert np.abs(g - prob.grad_shift(theta)).max() < TOL_E


# ------------------------------------------------------ packed sector layout

def _eval_layout(H, n, ne, theta, packed):
    """energy_grad with the packed layout on or off (fresh ansatz handle, so
    the plan is made under the requested setting)."""
    vq.set_packed(packed)
    try:
        return vq.energy_grad(H, vq.Ansatz.uccsd(n, ne), ne, theta)
    finally:
        vq.set_packed(True)


@pytest.mark.parametrize("n,ne", [(4, 2), (5, 2), (6, 3), (7, 3), (8, 4), (9, 5), (10, 5),
                                  (11, 4), (12, 6), (13, 7), (14, 7), (16, 8)])
def test_packed_layout_matches_full_layout_and_oracle(n, ne):
    """The packed sector layout (only in-sector amplitudes stored), with the
    string-product and the block-order H-apply, against full 2^n vectors and
    the oracle, odd and even n, open shells."""
    H, A, prob = _pair(n, ne, 1100 + n)
    theta = uniform_theta(1200 + n, A.n_params)
    ep, gp = _eval_layout(H, n, ne, theta, 2)
    eb, gb = _eval_layout(H, n, ne, theta, 1)
    ef, gf = _eval_layout(H, n, ne, theta, 0)
    assert abs(ep - ef) < 1e-12 and np.abs(gp - gf).max() < 1e-12
    assert abs(eb - ef) < 1e-12 and np.abs(gb - gf).max() < 1e-12
    assert abs(ep - prob.energy(theta)) < TOL_E
    idx = sorted(np.random.default_rng(n).choice(A.n_params, min(4, A.n_params),
                                                 replace=False).tolist())
    assert np.abs(gp[idx] - prob.grad_shift(theta, idx)).max() < TOL_E


@pytest.mark.parametrize("L", [6, 7, 9, 11, 12])
def test_packed_block_bits_agree(L):
    """Every block-bit count from the electron count up gives the same result
    (different block pairs, run splits and H-apply tiles)."""
    n, ne = 12, 6
    H, A, prob = _pair(n, ne, 1301)
    theta = uniform_theta(1302, A.n_params)
    lib = vq.lib()
    try:
        assert lib.vqe_set_tuning(n, 0, 65536, 65536, L) == 0
        e, g = vq.energy_grad(H, vq.Ansatz.uccsd(n, ne), ne, theta)
    finally:
        lib.vqe_set_tuning(n, 0, 0, 0, 0)
    ef, gf = _eval_layout(H, n, ne, theta, False)
    assert abs(e - prob.energy(theta)) < TOL_E
    assert abs(e - ef) < 1e-12 and np.abs(g - gf).max() < 1e-12


def test_packed_reference_only_programs():
    """Programs without excitations (closed shells ne = 0 and ne = n): the
    packed state is the reference alone."""
    for n, ne in [(6, 0), (6, 6), (5, 5)]:
        h0, h, g = random_integrals(n, 1400 + n)
        H = vq.Hamiltonian.from_integrals(n, h0, h, g)
        A = vq.Ansatz.uccsd(n, ne)
        assert A.n_params == 0
        e, grad = vq.energy_grad(H, A, ne, np.zeros(0))
        assert grad.size == 0
        assert abs(e - F.Problem(n, ne, h0, h, g).energy(np.zeros(0))) < TOL_E


def test_batch_packed_matches_full_layout():
    specs = [(8, 4, 1), (10, 5, 2), (11, 5, 3), (12, 6, 4), (12, 6, 5), (14, 7, 6)]
    Hs, thetas = [], []
    for n, ne, s in specs:
        h0, h, g = random_integrals(n, 1500 + s)
        Hs.append(vq.Hamiltonian.from_integrals(n, h0, h, g))
        thetas.append(uniform_theta(1600 + s, vq.Ansatz.uccsd(n, ne).n_params))
    flat = np.concatenate(thetas)
    out = []
    for packed in (2, 0):
        vq.set_packed(packed)
        try:
            b = vq.Batch(Hs, [vq.Ansatz.uccsd(n, ne) for n, ne, _ in specs],
                         [ne for _, ne, _ in specs])
        finally:
            vq.set_packed(True)
        out.append(b.energy_grad(flat))
    (e1, g1), (e2, g2) = out
    assert np.abs(e1 - e2).max() < 1e-12 and np.abs(g1 - g2).max() < 1e-12


@pytest.mark.parametrize("threads", [64, 256, 512, 1024])
def test_packed_run_thread_counts_agree(threads):
    """Every launch shape of the packed gate runs (threads per tile, entries
    per thread) gives the same energy and gradient."""
    n, ne = 14, 7
    H, A, prob = _pair(n, ne, 1701)
    theta = uniform_theta(1702, A.n_params)
    e0, g0 = vq.energy_grad(H, A, ne, theta)
    try:
        vq.set_run_threads(n, False, threads, threads)
        e, g = vq.energy_grad(H, vq.Ansatz.uccsd(n, ne), ne, theta)
    finally:
        vq.set_run_threads(n, False, 0, 0)
    assert abs(e - prob.energy(theta)) < TOL_E
    assert abs(e - e0) < 1e-12 and np.abs(g - g0).max() < 1e-12


def test_pair_lists_longer_than_the_block():
    """Gate runs whose pair lists are longer than the run's thread count (each
    thread then takes several pairs of a gate, the later ones read in the gate
    itself): 64-thread tiles of up to 1000 entries, against the oracle and
    the default launch shape."""
    n, ne = 16, 8
    H, A, prob = _pair(n, ne, 1711)
    theta = uniform_theta(1712, A.n_params)
    e0, g0 = vq.energy_grad(H, A, ne, theta)
    try:
        vq.set_run_threads(n, False, 64, 64)
        vq.set_tile_cap(n, False, 1000)
        e, g = vq.energy_grad(H, vq.Ansatz.uccsd(n, ne), ne, theta)
    finally:
        vq.set_run_threads(n, False, 0, 0)
        vq.set_tile_cap(n, False, 0)
    assert abs(e - prob.energy(theta)) < TOL_E
    k = [0, 1, A.n_params - 2, A.n_params - 1]
    assert np.abs(g[k] - prob.grad_shift(theta, k)).max() < TOL_E
    assert abs(e - e0) < 1e-12 and np.abs(g - g0).max() < 1e-12


def test_string_product_long_rows_match_block_order():
    """Beta-string rows longer than 256 take several waves per row in the
    string-product H-apply; against the block-order H-apply (itself pinned to
    the oracle above) at 22 qubits, 462 beta strings per row."""
    n, ne = 22, 10
    h0, h, g = random_integrals(n, 2201)
    H = vq.Hamiltonian.from_integrals(n, h0, h, g)
    theta = uniform_theta(2202, vq.Ansatz.uccsd(n, ne).n_params)
    e2, g2 = _eval_layout(H, n, ne, theta, 2)
    e1, g1 = _eval_layout(H, n, ne, theta, 1)
    assert abs(e2 - e1) < 1e-12 * max(1.0, abs(e1)) * 10
    assert np.abs(g2 - g1).max() < 1e-11


@pytest.mark.parametrize("n,ne", [(8, 4), (11, 5)])
def test_pair_records_off_the_chain_pattern(n, ne):
    """The string-product H-apply takes the beta signs of its alpha-beta pair
    records from the list entries when every record's mask is the chain
    between the pair's orbitals plus one mask per class (the Jordan-Wigner
    form), else from a per-pair mask.  Here every term of one alpha-beta
    double shape gets an extra Z on a beta qubit inside its chain (still
    Hermitian), which breaks that pattern: the packed path must match full
    vectors and the oracle's dense Pauli sums (energy and gradient)."""
    h0, h, g = random_integrals(n, 1300 + n)
    S = dict(P.jw_hamiltonian(n, h0, h, g))
    x0 = (1 << 0) | (1 << 2) | (1 << 3) | (1 << 7)   # alpha 0, 1 and beta 1, 3
    keys = [k for k in S if k[0] == x0]
    assert len(keys) >= 4 and all(k[1] & (1 << 5) for k in keys)   # beta 2 lies on the chain
    for k in keys:
        S[(k[0], k[1] ^ (1 << 5))] = S.pop(k)
    fold = P.folded_terms(S)   # the boundary's real form c i^{#Y} X^x Z^z
    H = vq.Hamiltonian.from_paulis(n, np.array([k[0] for k in fold], np.uint32),
                                   np.array([k[1] for k in fold], np.uint32),
                                   np.array(list(fold.values())))
    A = vq.Ansatz.uccsd(n, ne)
    excs = F.uccsd_excitations(n, ne)
    theta = uniform_theta(n + 40, A.n_params, -0.4, 0.4)
    out = {}
    try:
        for mode in (2, 0):
            vq.set_packed(mode)
            out[mode] = vq.energy_grad(H, A, ne, theta)
    finally:
        vq.set_packed(2)
    e_or = P.energy(S, P.prepare(n, ne, excs, theta), n)
    assert abs(out[2][0] - e_or) < TOL_E and abs(out[0][0] - e_or) < TOL_E
    assert np.abs(out[2][1] - out[0][1]).max() < TOL_E
    # the altered terms matter
    e_jw = P.energy(P.jw_hamiltonian(n, h0, h, g), P.prepare(n, ne, excs, theta), n)
    assert abs(e_or - e_jw) > 1e-6
    # sampled gradient components against the oracle's shift rule
    c2 = (math.sqrt(2.0) - 1.0) / 2.0
    for j in (0, A.n_params // 2, A.n_params - 1):
        def e(d):
            t = theta.copy()
            t[j] += d
            return P.energy(S, P.prepare(n, ne, excs, t), n)
        gj = (e(math.pi / 4) - e(-math.pi / 4)) - c2 * (e(math.pi / 2) - e(-math.pi / 2))
        assert abs(out[2][1][j] - gj) < TOL_E


@pytest.mark.parametrize("k", [0, 5, 10, 15, 19])
def test_scan12_geometries_match_oracle_and_fd(k):
    """The 12-qubit bond-stretch family (20 geometries, one batch as bench.py
    runs it): at every fifth geometry the energy and every gradient component
    against the oracle (four-term shift rule, 1e-10), and every component
    against central differences of the GPU energy (h = 1e-5, 1e-6)."""
    from vqe_inputs import SCAN12_LAMBDAS
    fam = scan_integrals(12, 2)
    A = vq.Ansatz.uccsd(12, 6)
    Hs = [vq.Hamiltonian.from_integrals(12, *fam(l)) for l in SCAN12_LAMBDAS]
    theta = uniform_theta(7, A.n_params)
    b = vq.Batch(Hs, [A] * len(Hs), [6] * len(Hs))
    e, g = b.energy_grad(np.concatenate([theta] * len(Hs)))
    M = A.n_params
    gk = g[k * M:(k + 1) * M]
    prob = F.Problem(12, 6, *fam(SCAN12_LAMBDAS[k]))
    assert abs(e[k] - prob.energy(theta)) < TOL_E
    assert np.abs(gk - prob.grad_shift(theta)).max() < TOL_E
    fd = np.empty(M)
    for j in range(M):
        tp, tm = theta.copy(), theta.copy()
        tp[j] += 1e-5
        tm[j] -= 1e-5
        fd[j] = (vq.energy_grad(Hs[k], A, 6, tp, grad=False)[0] -
                 vq.energy_grad(Hs[k], A, 6, tm, grad=False)[0]) / 2e-5
    assert np.abs(gk - fd).max() < 1e-6
