"""The allocation-free energy + gradient entry point (its workspace is a
static device array; plans come from a prior vqe_energy_grad) against
vqe_energy_grad on the same inputs: the packed sector layout, the
full-vector sector layout (lambda must be cleared in the shared array) and a
Pauli-rotation program on full vectors; two calls in a row with the second
smaller; the errors for a missing set-up and an oversize problem; and device
free memory unchanged across calls."""
import numpy as np
import pytest

import paper_2311_01242_amd as vq
from vqe_inputs import random_integrals, uniform_theta

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield


def _problem(n, ne, seed):
    h0, h, g = random_integrals(n, seed)
    return vq.Hamiltonian.from_integrals(n, h0, h, g), vq.Ansatz.uccsd(n, ne)


def _check_pair(H, A, ne, theta):
    e0, g0 = vq.energy_grad(H, A, ne, theta)            # set-up (builds the plans)
    e1, g1 = vq.energy_grad_noalloc(H, A, ne, theta)
    assert abs(e1 - e0) < TOL and np.abs(g1 - g0).max() < TOL
    e2, none = vq.energy_grad_noalloc(H, A, ne, theta, grad=False)
    assert none is None and abs(e2 - e0) < TOL
    return e1, g1


def test_two_calls_second_smaller_packed():
    H16, A16 = _problem(16, 8, 901)
    H12, A12 = _problem(12, 6, 902)
    t16 = uniform_theta(903, A16.n_params, -0.3, 0.3)
    t12 = uniform_theta(904, A12.n_params, -0.3, 0.3)
    _check_pair(H16, A16, 8, t16)
    _check_pair(H12, A12, 6, t12)
    # and the larger one again after the smaller
    _check_pair(H16, A16, 8, t16)


def test_full_vector_layouts_after_other_contents():
    # a Pauli-rotation program (full vectors, lambda fully written) first
    n = 10
    h0, h, g = random_integrals(n, 905)
    H = vq.Hamiltonian.from_integrals(n, h0, h, g)
    rng = np.random.default_rng(906)
    x = rng.integers(1, 1 << n, 40).astype(np.uint32)
    z = rng.integers(0, 1 << n, 40).astype(np.uint32)
    R = vq.Ansatz.from_rotations(n, 40, x, z, np.arange(40, dtype=np.int32), np.ones(40))
    _check_pair(H, R, 5, rng.uniform(-1, 1, 40))
    # then UCCSD on full 2^n vectors (sector H-apply: lambda must start at zero)
    try:
        vq.set_packed(0)
        H2, A2 = _problem(n, 5, 907)
        _check_pair(H2, A2, 5, uniform_theta(908, A2.n_params, -0.3, 0.3))
    finally:
        vq.set_packed(2)


def test_missing_setup_and_oversize_are_rejected():
    H, A = _problem(12, 6, 909)
    theta = uniform_theta(910, A.n_params)
    with pytest.raises(vq.VQEError) as ex:
        vq.energy_grad_noalloc(H, A, 6, theta)
    assert ex.value.code == vq.VQE_EINVAL
    # full vectors at 22 qubits: phi and lambda alone (2 x 2^22 complex
    # amplitudes, 128 MiB) exceed the 64 MiB scratch, whatever the tiling
    vq.set_packed(0)
    try:
        H22, A22 = _problem(22, 11, 911)
        t22 = uniform_theta(912, A22.n_params)
        vq.energy_grad(H22, A22, 11, t22, grad=False)        # plans exist now
        with pytest.raises(vq.VQEError) as ex:
            vq.energy_grad_noalloc(H22, A22, 11, t22)
        assert ex.value.code == vq.VQE_ERANGE and "scratch" in str(ex.value)
    finally:
        vq.set_packed(True)


def test_device_memory_unchanged_across_calls():
    import torch
    H, A = _problem(14, 7, 913)
    theta = uniform_theta(914, A.n_params)
    vq.energy_grad(H, A, 7, theta)
    vq.energy_grad_noalloc(H, A, 7, theta)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for _ in range(20):
        vq.energy_grad_noalloc(H, A, 7, theta)
    torch.cuda.synchronize()
    assert torch.cuda.mem_get_info()[0] == free0
