"""GPU parity of the Bravyi-Kitaev mapping (Sec. 2.1.1): the BK Hamiltonian
and the BK-encoded UCCSD rotations on full 2^n vectors from the encoded
reference, against the oracle (energies are mapping independent, so the
CI-space oracle applies directly; the statevector against the oracle's own
Fenwick-set BK evolution).  Tolerance 1e-10 Ha."""
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


@pytest.fixture(params=[0, 2], ids=["full-vector-rotations", "packed-occupation-basis"])
def layout(request):
    """BK programs as encoded Pauli rotations on full vectors, and (the
    default) in the occupation basis on the packed sector path."""
    vq.set_packed(request.param)
    yield request.param
    vq.set_packed(True)


@pytest.mark.parametrize("n,ne", [(4, 2), (5, 2), (6, 3), (8, 4), (10, 5), (12, 6), (13, 6)])
def test_bk_energy_and_gradient_vs_oracle(n, ne, layout):
    h0, h, g = random_integrals(n, 1000 + n)
    H = vq.Hamiltonian.from_integrals_map(n, "bk", h0, h, g)
    A = vq.Ansatz.uccsd_map(n, ne, "bk")
    prob = F.Problem(n, ne, h0, h, g)
    theta = uniform_theta(n, A.n_params, -0.4, 0.4)
    e, gr = vq.energy_grad(H, A, ne, theta)
    assert abs(e - prob.energy(theta)) < TOL_E
    assert np.abs(gr - prob.grad_shift(theta)).max() < TOL_E
    e0, g0 = vq.energy_grad(H, A, ne, np.zeros(A.n_params))
    assert abs(e0 - F.hf_energy_closed_form(n, ne, h0, h, g)) < TOL_E
    # the allocation-free call reuses the plan of the call before it
    e1, g1 = vq.energy_grad_noalloc(H, A, ne, np.zeros(A.n_params))
    assert e1 == e0 and np.array_equal(g1, g0)


def test_bk_layouts_agree_on_a_batch():
    """A 12-qubit BK stretch batch: occupation-basis packed evaluation against
    the encoded rotations on full vectors (1e-12), and the Hamiltonian's
    terms taken to the occupation basis against the Jordan-Wigner ones."""
    fam = scan_integrals(12, 5)
    lams = np.linspace(0.8, 2.5, 5)
    A = vq.Ansatz.uccsd_map(12, 6, "bk")
    th = np.concatenate([uniform_theta(70 + i, A.n_params, -0.3, 0.3) for i in range(len(lams))])
    out = []
    for mode in (0, 2):
        vq.set_packed(mode)
        try:
            Hs = [vq.Hamiltonian.from_integrals_map(12, "bk", *fam(l)) for l in lams]
            b = vq.Batch(Hs, [A] * len(Hs), [6] * len(Hs))
            out.append(b.energy_grad(th))
        finally:
            vq.set_packed(True)
    (e0, g0), (e2, g2) = out
    assert np.abs(e0 - e2).max() < 1e-12 and np.abs(g0 - g2).max() < 1e-12
    # the same values as the Jordan-Wigner program on the same integrals
    Aj = vq.Ansatz.uccsd(12, 6)
    bj = vq.Batch([vq.Hamiltonian.from_integrals(12, *fam(l)) for l in lams], [Aj] * len(lams),
                  [6] * len(lams))
    ej, gj = bj.energy_grad(th)
    assert np.abs(ej - e2).max() < 1e-12 and np.abs(gj - g2).max() < 1e-12


def test_bk_statevector_matches_oracle():
    import torch
    n, ne = 8, 4
    A = vq.Ansatz.uccsd_map(n, ne, "bk")
    theta = uniform_theta(3, A.n_params, -0.5, 0.5)
    t = torch.empty(1 << n, dtype=torch.complex128, device="cuda")
    s = vq.State.wrap(t)
    s.prepare_basis(A.reference())
    s.apply_ansatz(A, theta)
    torch.cuda.synchronize()
    ref = P.prepare(n, ne, F.uccsd_excitations(n, ne), theta, mapping="bk")
    assert np.abs(t.cpu().numpy() - ref).max() < 1e-12


def test_bk_vqe_matches_jw_4q():
    n, ne = 4, 2
    h0, h, g = random_integrals(n, 2)
    fci = F.Problem(n, ne, h0, h, g).fci()
    for mapping in ("jw", "bk"):
        H = vq.Hamiltonian.from_integrals_map(n, mapping, h0, h, g)
        A = vq.Ansatz.uccsd_map(n, ne, mapping)
        _, res, _ = vq.run_vqe(H, A, ne, max_iter=100, gtol=1e-10)
        assert abs(res.energy - fci) < 1e-9


def test_bk_batch_matches_single():
    fam = scan_integrals(10, 3)
    lams = np.linspace(0.8, 2.5, 6)
    Hs = [vq.Hamiltonian.from_integrals_map(10, "bk", *fam(l)) for l in lams]
    A = vq.Ansatz.uccsd_map(10, 5, "bk")
    b = vq.Batch(Hs, [A] * len(Hs), [5] * len(Hs))
    th = np.concatenate([uniform_theta(60 + i, A.n_params) for i in range(len(Hs))])
    e, g = b.energy_grad(th)
    m = A.n_params
    for i in range(len(Hs)):
        e1, g1 = vq.energy_grad(Hs[i], A, 5, th[m * i:m * (i + 1)])
        assert abs(e[i] - e1) < 1e-12
        assert np.abs(g[m * i:m * (i + 1)] - g1).max() < 1e-12
    prob = F.Problem(10, 5, *fam(lams[2]))
    assert abs(e[2] - prob.energy(th[2 * m:3 * m])) < TOL_E
