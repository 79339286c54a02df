"""Real amplitudes on the string-product path against complex amplitudes:
the same energies and gradients (to rounding) for single states, batches of
several size classes, the allocation-free call's plan and ADAPT pool
gradients; and the real path against the oracle.  Excitation gates are real
rotations and the Hamiltonian is a real matrix, so phi = U|HF> and H phi are
real (Sec. 2.1.2, Eq. 2)."""
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
    yield
    vq.set_real(True)


def _both(fn):
    out = []
    for real in (False, True):
        vq.set_real(real)
        try:
            out.append(fn())
        finally:
            vq.set_real(True)
    return out


@pytest.mark.parametrize("n,ne", [(4, 2), (8, 4), (11, 5), (14, 7), (17, 8), (20, 10)])
def test_single_state_real_equals_complex(n, ne):
    h0, h, g = random_integrals(n, 9100 + n)
    # new handles per mode: plans are cached per (ansatz, device) when made
    def run():
        H = vq.Hamiltonian.from_integrals(n, h0, h, g)
        A = vq.Ansatz.uccsd(n, ne)
        th = uniform_theta(9200 + n, A.n_params, -0.3, 0.3)
        return vq.energy_grad(H, A, ne, th)
    (ec, gc), (er, gr) = _both(run)
    assert abs(ec - er) < 1e-12
    assert np.abs(gc - gr).max() < 1e-12
    if n <= 14:
        A = vq.Ansatz.uccsd(n, ne)
        th = uniform_theta(9200 + n, A.n_params, -0.3, 0.3)
        prob = F.Problem(n, ne, h0, h, g)
        assert abs(er - prob.energy(th)) < TOL_E
        k = min(4, A.n_params)
        assert np.abs(gr[:k] - prob.grad_shift(th, range(k))).max() < TOL_E


def test_batch_real_equals_complex():
    sizes = [12, 13, 14, 15, 16, 17, 18, 12, 16]
    ints = [random_integrals(n, 9300 + i) for i, n in enumerate(sizes)]

    def run():
        Hs = [vq.Hamiltonian.from_integrals(n, *ints[i]) for i, n in enumerate(sizes)]
        As = [vq.Ansatz.uccsd(n, n // 2) for n in sizes]
        b = vq.Batch(Hs, As, [n // 2 for n in sizes])
        th = np.concatenate([uniform_theta(9400 + i, a.n_params, -0.2, 0.2) for i, a in enumerate(As)])
        e, g = b.energy_grad(th)
        e2, g2 = b.energy_grad(th)
        assert np.array_equal(e, e2) and np.array_equal(g, g2)   # replays are bitwise stable
        return e, g
    (ec, gc), (er, gr) = _both(run)
    assert np.abs(ec - er).max() < 1e-12
    assert np.abs(gc - gr).max() < 1e-12


def test_pool_gradient_real_equals_complex():
    n, ne = 12, 6
    h0, h, g = random_integrals(n, 9500)

    def run():
        H = vq.Hamiltonian.from_integrals(n, h0, h, g)
        pool = vq.Ansatz.uccsd(n, ne)
        A = pool.select([3, 40, 7, 100])
        th = uniform_theta(9501, A.n_params, -0.4, 0.4)
        return vq.pool_gradient(H, A, pool, ne, th)
    (ec, gc), (er, gr) = _both(run)
    assert abs(ec - er) < 1e-12
    assert np.abs(gc - gr).max() < 1e-12


def test_noalloc_real_equals_complex():
    n, ne = 14, 7
    h0, h, g = random_integrals(n, 9600)

    def run():
        H = vq.Hamiltonian.from_integrals(n, h0, h, g)
        A = vq.Ansatz.uccsd(n, ne)
        th = uniform_theta(9601, A.n_params, -0.3, 0.3)
        e1, g1 = vq.energy_grad(H, A, ne, th)
        e2, g2 = vq.energy_grad_noalloc(H, A, ne, th)
        assert e1 == e2 and np.array_equal(g1, g2)
        return e2, g2
    (ec, gc), (er, gr) = _both(run)
    assert abs(ec - er) < 1e-12
    assert np.abs(gc - gr).max() < 1e-12
