"""GPU parity of pUCCD in the hard-core-boson form (Sec. 2.1, ansatz list):
the pair Hamiltonian and pair Givens program through the C ABI against the
oracle's pair-space energies and shift-rule gradients (1e-10 Ha), the
batch against the single-state path, and VQE against the oracle's minimum."""
import numpy as np
import pytest

import paper_2311_01242_amd as vq
from oracle import hcb as HB
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


def _pair(n_orb, n_pairs, seed):
    h0, h, g = random_integrals(2 * n_orb, seed)
    return (vq.Hamiltonian.pairs_from_integrals(n_orb, h0, h, g), vq.Ansatz.puccd(n_orb, n_pairs),
            HB.Problem(n_orb, n_pairs, h0, h, g))


@pytest.mark.parametrize("n_orb,n_pairs", [(2, 1), (3, 1), (4, 2), (5, 3), (6, 2), (7, 3), (9, 4),
                                           (11, 7), (12, 6)])
def test_energy_and_gradient_vs_oracle(n_orb, n_pairs):
    H, A, prob = _pair(n_orb, n_pairs, 300 + n_orb)
    theta = uniform_theta(n_orb, A.n_params, -0.6, 0.6)
    e, g = vq.energy_grad(H, A, n_pairs, theta)
    assert abs(e - prob.energy(theta)) < TOL_E
    assert np.abs(g - prob.grad_shift(theta)).max() < TOL_E
    e0, g0 = vq.energy_grad(H, A, n_pairs, np.zeros(A.n_params))
    assert abs(e0 - prob.energy(np.zeros(A.n_params))) < TOL_E


def test_statevector_matches_oracle():
    n_orb, n_pairs = 8, 4
    H, A, prob = _pair(n_orb, n_pairs, 5)
    theta = uniform_theta(9, A.n_params, -1.0, 1.0)
    import torch
    t = torch.empty(1 << n_orb, dtype=torch.complex128, device="cuda")
    s = vq.State.wrap(t)
    s.prepare_hf(n_pairs)
    s.apply_ansatz(A, theta)
    torch.cuda.synchronize()
    got = t.cpu().numpy()
    ref = prob.space.to_statevector(prob.state(theta))
    assert np.abs(got - ref).max() < 1e-12


def test_vqe_reaches_oracle_minimum():
    n_orb, n_pairs = 6, 3
    H, A, prob = _pair(n_orb, n_pairs, 12)
    theta, res, _ = vq.run_vqe(H, A, n_pairs, max_iter=300, gtol=1e-9)
    import scipy.optimize
    ref = scipy.optimize.minimize(lambda t: (prob.energy(t), prob.grad_shift(t)),
                                  np.zeros(prob.n_params), jac=True, method="BFGS",
                                  options={"gtol": 1e-10})
    assert res.converged == 1
    assert abs(res.energy - ref.fun) < 1e-9
    assert np.abs(prob.grad_shift(theta)).max() < 1e-7
    assert res.energy >= prob.ground() - 1e-10


def test_batch_matches_single_on_a_stretch_scan():
    """The CH3F-sized pair problem (11 orbitals, 7 pairs, 28 parameters) along
    a stretch family, batched in one graph, against single evaluations and
    sampled oracle values."""
    fam = scan_integrals(22, 8)
    lams = np.linspace(0.8, 2.5, 24)
    Hs = [vq.Hamiltonian.pairs_from_integrals(11, *fam(l)) for l in lams]
    A = vq.Ansatz.puccd(11, 7)
    assert A.n_params == 28
    b = vq.Batch(Hs, [A] * len(Hs), [7] * len(Hs))
    th = np.concatenate([uniform_theta(100 + i, 28, -0.3, 0.3) for i in range(len(Hs))])
    e, g = b.energy_grad(th)
    for i in range(len(Hs)):
        e1, g1 = vq.energy_grad(Hs[i], A, 7, th[28 * i:28 * (i + 1)])
        assert abs(e[i] - e1) < 1e-12
        assert np.abs(g[28 * i:28 * (i + 1)] - g1).max() < 1e-12
    for i in (0, 11, 23):
        prob = HB.Problem(11, 7, *fam(lams[i]))
        t = th[28 * i:28 * (i + 1)]
        assert abs(e[i] - prob.energy(t)) < TOL_E
        assert np.abs(g[28 * i:28 * (i + 1)] - prob.grad_shift(t)).max() < TOL_E
