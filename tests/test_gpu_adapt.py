"""GPU parity of ADAPT-VQE (Sec. 2.1, "ADAPT-VQE algorithm"): operator
selection, the pool gradient (one reverse sweep of the pool at angle zero
after the forward pass and H-apply) and the growth loop, through the C ABI,
against the CPU oracle's shift-rule pool gradient and its own ADAPT loop.
Tolerance 1e-10 Ha for energies and gradients (FP64 on both sides)."""
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


def _setup(n, ne, seed):
    h0, h, g = random_integrals(n, seed)
    return vq.Hamiltonian.from_integrals(n, h0, h, g), vq.Ansatz.uccsd(n, ne), (h0, h, g)


def _oracle(n, ne, ints, sel):
    pool = F.uccsd_excitations(n, ne)
    return F.Problem(n, ne, *ints, excs=[pool[k] for k in sel]), pool


@pytest.mark.parametrize("n,ne", [(4, 2), (6, 3), (9, 4), (12, 6)])
def test_select_matches_oracle(n, ne):
    H, pool, ints = _setup(n, ne, 40 + n)
    rng = np.random.default_rng(n)
    sel = [int(k) for k in rng.integers(0, pool.n_params, 7)]
    sel.append(sel[2])                                   # an operator used twice
    A = pool.select(sel)
    assert A.n_params == len(sel)
    assert A.excitations() == [tuple(pool.excitations()[k]) for k in sel]
    prob, _ = _oracle(n, ne, ints, sel)
    theta = uniform_theta(n, len(sel), -0.5, 0.5)
    e, g = vq.energy_grad(H, A, ne, theta)
    assert abs(e - prob.energy(theta)) < TOL_E
    assert np.abs(g - prob.grad_shift(theta)).max() < TOL_E


@pytest.mark.parametrize("n,ne", [(4, 2), (8, 4), (13, 6)])
def test_identity_program_is_hf(n, ne):
    H, pool, ints = _setup(n, ne, 50 + n)
    A = pool.select([])
    assert A.n_params == 0
    e, g = vq.pool_gradient(H, A, pool, ne, np.zeros(0))
    assert abs(e - F.hf_energy_closed_form(n, ne, *ints)) < TOL_E
    assert np.abs(g - F.grad_at_hf_closed_form(ne, F.uccsd_excitations(n, ne), ints[1], ints[2])).max() < TOL_E


@pytest.mark.parametrize("mode", [2, 1, 0])
@pytest.mark.parametrize("n,ne,k", [(4, 2, 2), (6, 3, 5), (9, 4, 6), (12, 6, 9), (13, 6, 4), (14, 7, 12)])
def test_pool_gradient_vs_oracle(mode, n, ne, k):
    """All three layouts: packed string-product, packed block order, full 2^n."""
    vq.set_packed(mode)
    try:
        H, pool, ints = _setup(n, ne, 60 + n)
        rng = np.random.default_rng(100 + n)
        sel = [int(v) for v in rng.integers(0, pool.n_params, k)]
        theta = rng.uniform(-0.6, 0.6, k)
        A = pool.select(sel)
        e, g = vq.pool_gradient(H, A, pool, ne, theta)
        prob, plist = _oracle(n, ne, ints, sel)
        e_ref, g_ref = F.pool_gradient(prob, theta, plist)
        assert abs(e - e_ref) < TOL_E
        assert np.abs(g - g_ref).max() < TOL_E
        # the energy half agrees with the plain evaluation
        assert abs(e - vq.energy_grad(H, A, ne, theta, grad=False)[0]) < 1e-12
    finally:
        vq.set_packed(2)


def test_pool_gradient_of_last_operator_is_its_own_gradient():
    """Appending the ansatz's last operator again only adds to its angle."""
    n, ne = 12, 6
    H, pool, _ = _setup(n, ne, 77)
    sel = [3, 50, 11, 90]
    A = pool.select(sel)
    theta = uniform_theta(5, len(sel), -0.4, 0.4)
    _, gp = vq.pool_gradient(H, A, pool, ne, theta)
    _, g = vq.energy_grad(H, A, ne, theta)
    assert abs(gp[90] - g[-1]) < 1e-12


def test_pool_gradient_rejects_mismatch():
    H, pool, _ = _setup(8, 4, 1)
    other = vq.Ansatz.uccsd(8, 2)
    with pytest.raises(vq.VQEError):
        vq.pool_gradient(H, pool.select([0]), other, 4, np.zeros(1))
    with pytest.raises(vq.VQEError):
        pool.select([pool.n_params])


@pytest.mark.parametrize("n,ne,seed", [(4, 2, 1), (4, 2, 2), (6, 3, 3), (6, 4, 4)])
def test_adapt_matches_oracle_loop(n, ne, seed):
    """Same operator sequence, energies and gradient norms as the oracle's
    ADAPT loop; every selection in these cases is separated from the runner-up
    by far more than the two sides' rounding (checked on the oracle side)."""
    h0, h, g = random_integrals(n, seed)
    H = vq.Hamiltonian.from_integrals(n, h0, h, g)
    pool = vq.Ansatz.uccsd(n, ne)
    sel, th, es, ns, res = vq.run_adapt(H, pool, ne, grad_tol=1e-5, max_iter=400, gtol=1e-9)
    steps = []
    sel_r, th_r, es_r, ns_r = F.adapt(n, ne, h0, h, g, grad_tol=1e-5, gtol=1e-9, record=steps)
    # well-posed selections: the pick beats every non-tied operator clearly
    for _, gp in steps[:-1]:
        mag = np.abs(gp)
        top = mag.max()
        assert np.all((mag >= top - 1e-10) | (mag <= top - 1e-6))
    assert sel == sel_r
    assert res.converged == 1 and res.n_operators == len(sel)
    assert np.abs(es - es_r).max() < 1e-9
    assert np.abs(ns - ns_r).max() < 1e-5
    assert abs(res.energy - es[-1]) == 0.0


@pytest.mark.parametrize("n,ne,cap", [(8, 4, 10), (12, 6, 8)])
def test_adapt_trace_replayed_on_oracle(n, ne, cap):
    """The GPU loop's final angles checked on the oracle (energy, stationarity),
    its energies never rising, and each step replayed on the oracle along the
    GPU's operator sequence (the oracle re-optimising the angles itself): the
    pool-gradient norm, that the pick is a largest |gradient|, and the
    energy after the re-optimisation."""
    h0, h, g = random_integrals(n, 500 + n)
    H = vq.Hamiltonian.from_integrals(n, h0, h, g)
    pool = vq.Ansatz.uccsd(n, ne)
    sel, th, es, ns, res = vq.run_adapt(H, pool, ne, grad_tol=1e-6, max_operators=cap,
                                        max_iter=400, gtol=1e-9)
    assert res.n_operators == cap and res.converged == 0
    plist = F.uccsd_excitations(n, ne)
    A = pool.select(sel)
    e_fin, _ = vq.energy_grad(H, A, ne, th)
    assert abs(e_fin - es[-1]) < 1e-12
    prob = F.Problem(n, ne, h0, h, g, excs=[plist[i] for i in sel])
    assert abs(prob.energy(th) - es[-1]) < TOL_E
    assert np.abs(prob.grad_shift(th)).max() < 1e-7
    assert np.all(np.diff(es) <= 1e-12)
    # the picks, at the angles the loop held before each one
    prev = np.zeros(0)
    for k in range(cap):
        sub = F.Problem(n, ne, h0, h, g, excs=[plist[i] for i in sel[:k]])
        _, gp = F.pool_gradient(sub, prev, plist)
        assert abs(np.linalg.norm(gp) - ns[k]) < 1e-7
        assert abs(gp[sel[k]]) >= np.abs(gp).max() - 1e-7
        run = F.Problem(n, ne, h0, h, g, excs=[plist[i] for i in sel[:k + 1]])
        prev = run.vqe(theta0=np.append(prev, 0.0), gtol=1e-10, maxiter=400).x
        assert abs(run.energy(prev) - es[k + 1]) < 1e-8
