"""GPU parity of the deeper UCC ansatze of Sec. 2.1's ansatz list: UCCSD with
several Trotter steps (shared angles) and k-UpCCGSD (generalised singles and
pair doubles, k layers), in all three layouts, against the oracle (1e-10 Ha).
Generalised excitations may annihilate orbitals above the packed block bits:
those gates pair blocks h and (h minus the annihilated high bits) plus the
created ones, which the 18-qubit cases exercise for every block size."""
import numpy as np
import pytest

import paper_2311_01242_amd as vq
from oracle import fermion as F
from vqe_inputs import random_integrals, uniform_theta

pytestmark = pytest.mark.gpu

TOL_E = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    vq.set_packed(2)
    yield
    vq.set_packed(2)


@pytest.mark.parametrize("mode", [2, 1, 0])
@pytest.mark.parametrize("n,ne,steps", [(4, 2, 2), (6, 3, 3), (9, 4, 2), (12, 6, 2)])
def test_trotter_uccsd_vs_oracle(mode, n, ne, steps):
    vq.set_packed(mode)
    try:
        h0, h, g = random_integrals(n, 700 + n)
        H = vq.Hamiltonian.from_integrals(n, h0, h, g)
        A = vq.Ansatz.uccsd_trotter(n, ne, steps)
        tp = F.TrotterProblem(n, ne, h0, h, g, steps)
        theta = uniform_theta(n + steps, A.n_params, -0.5, 0.5)
        e, gr = vq.energy_grad(H, A, ne, theta)
        assert abs(e - tp.energy(theta)) < TOL_E
        assert np.abs(gr - tp.grad(theta)).max() < TOL_E
    finally:
        vq.set_packed(2)


@pytest.mark.parametrize("mode", [2, 1, 0])
@pytest.mark.parametrize("n,ne,k", [(4, 2, 1), (4, 2, 2), (6, 3, 2), (9, 4, 1), (12, 6, 2), (14, 7, 1)])
def test_kupccgsd_vs_oracle(mode, n, ne, k):
    vq.set_packed(mode)
    try:
        h0, h, g = random_integrals(n, 800 + n)
        H = vq.Hamiltonian.from_integrals(n, h0, h, g)
        A = vq.Ansatz.kupccgsd(n, ne, k)
        prob = F.Problem(n, ne, h0, h, g, excs=F.kupccgsd_excitations(n, k))
        theta = uniform_theta(n + 10 * k, A.n_params, -0.5, 0.5)
        e, gr = vq.energy_grad(H, A, ne, theta)
        assert abs(e - prob.energy(theta)) < TOL_E
        assert np.abs(gr - prob.grad_shift(theta)).max() < TOL_E
    finally:
        vq.set_packed(2)


@pytest.mark.parametrize("n,ne,k", [(17, 8, 1), (18, 9, 2)])
def test_kupccgsd_high_annihilated_orbitals(n, ne, k):
    """Packed layout (gates whose annihilated orbitals lie above the block
    bits) against full 2^n vectors, and sampled oracle values."""
    h0, h, g = random_integrals(n, 900 + n)
    H = vq.Hamiltonian.from_integrals(n, h0, h, g)
    A = vq.Ansatz.kupccgsd(n, ne, k)
    theta = uniform_theta(n, A.n_params, -0.3, 0.3)
    vq.set_packed(2)
    e2, g2 = vq.energy_grad(H, A, ne, theta)
    vq.set_packed(1)
    e1, g1 = vq.energy_grad(H, A, ne, theta)
    vq.set_packed(0)
    try:
        e0, g0 = vq.energy_grad(H, A, ne, theta)
    finally:
        vq.set_packed(2)
    assert abs(e2 - e0) < TOL_E and abs(e1 - e0) < TOL_E
    assert np.abs(g2 - g0).max() < TOL_E and np.abs(g1 - g0).max() < TOL_E
    prob = F.Problem(n, ne, h0, h, g, excs=F.kupccgsd_excitations(n, k))
    assert abs(e2 - prob.energy(theta)) < TOL_E
    # gradient components of gates with high annihilated orbitals, and others
    excs = F.kupccgsd_excitations(n, k)
    high = [j for j, x in enumerate(excs) if min(x[:len(x) // 2]) >= 14]
    assert high, "no gate annihilates above bit 13"
    idx = [0, high[0], high[-1], len(excs) - 1]
    ref = prob.grad_shift(theta, idx=idx)
    assert np.abs(g2[idx] - ref).max() < TOL_E


def test_kupccgsd_vqe_4q_reaches_fci():
    n, ne = 4, 2
    h0, h, g = random_integrals(n, 9)
    H = vq.Hamiltonian.from_integrals(n, h0, h, g)
    A = vq.Ansatz.kupccgsd(n, ne, 2)
    th0 = uniform_theta(2, A.n_params, -0.1, 0.1)
    theta, res, _ = vq.run_vqe(H, A, ne, theta0=th0, max_iter=300, gtol=1e-9)
    fci = F.Problem(n, ne, h0, h, g).fci()
    assert res.energy >= fci - 1e-10
    assert abs(res.energy - fci) < 1e-7


def test_adapt_over_a_generalised_pool():
    """ADAPT with the k-UpCCGSD layer as its pool (gates that annihilate
    virtual orbitals included) against the oracle's pool gradients."""
    n, ne = 8, 4
    h0, h, g = random_integrals(n, 61)
    H = vq.Hamiltonian.from_integrals(n, h0, h, g)
    pool = vq.Ansatz.kupccgsd(n, ne, 1)
    plist = F.kupccgsd_layer(n)
    sel = [3, 17, 0, 12]
    theta = uniform_theta(4, len(sel), -0.5, 0.5)
    e, gp = vq.pool_gradient(H, pool.select(sel), pool, ne, theta)
    prob = F.Problem(n, ne, h0, h, g, excs=[plist[i] for i in sel])
    e_ref, g_ref = F.pool_gradient(prob, theta, plist)
    assert abs(e - e_ref) < TOL_E
    assert np.abs(gp - g_ref).max() < TOL_E
