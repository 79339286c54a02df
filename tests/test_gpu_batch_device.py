"""The batch evaluation on device-resident buffers against the host-buffer
entry: the same energies and the same gradient bits for every kind of size
class a batch can hold (packed UCCSD of several qubit counts, the pUCCD pair
sector, Bravyi-Kitaev rotation programs on full vectors), on consecutive calls
with new parameters written on the caller's stream just before each call, and
against the oracle on sampled states."""
import numpy as np
import pytest

import paper_2311_01242_amd as vq
from oracle import fermion as F
from oracle import hcb as HB
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


def _mixed():
    Hs, As, nes, thetas, checks = [], [], [], [], []
    for i, n in enumerate([4, 8, 12, 14, 12, 16]):
        ne = n // 2
        h0, h, g = random_integrals(n, 8100 + i)
        Hs.append(vq.Hamiltonian.from_integrals(n, h0, h, g))
        As.append(vq.Ansatz.uccsd(n, ne))
        nes.append(ne)
        thetas.append(uniform_theta(8200 + i, As[-1].n_params, -0.3, 0.3))
        checks.append(("f", len(Hs) - 1, F.Problem(n, ne, h0, h, g)))
    for i in range(3):
        h0, h, g = random_integrals(22, 8300 + i)
        Hs.append(vq.Hamiltonian.pairs_from_integrals(11, h0, h, g))
        As.append(vq.Ansatz.puccd(11, 7))
        nes.append(7)
        thetas.append(uniform_theta(8400 + i, 28, -0.5, 0.5))
        checks.append(("p", len(Hs) - 1, HB.Problem(11, 7, h0, h, g)))
    h0, h, g = random_integrals(8, 8500)
    Hs.append(vq.Hamiltonian.from_integrals_map(8, "bk", h0, h, g))
    As.append(vq.Ansatz.uccsd_map(8, 4, "bk"))
    nes.append(4)
    thetas.append(uniform_theta(8600, As[-1].n_params, -0.3, 0.3))
    return Hs, As, nes, thetas, checks


def test_device_entry_matches_host_entry_bitwise():
    import torch
    Hs, As, nes, thetas, checks = _mixed()
    b = vq.Batch(Hs, As, nes)
    flat = np.concatenate(thetas)
    P = int(b.offsets[-1])
    th = torch.empty(P, dtype=torch.float64, device="cuda")
    e = torch.empty(b.S, dtype=torch.float64, device="cuda")
    g = torch.empty(P, dtype=torch.float64, device="cuda")
    for scale in (1.0, 0.5, -0.25):
        # written on the caller's stream just before the call: the batch
        # orders its evaluation after it
        th.copy_(torch.from_numpy(flat * scale).to("cuda", non_blocking=False))
        th.mul_(1.0)
        b.energy_grad_device(th, e, g)
        e_d, g_d = e.cpu().numpy(), g.cpu().numpy()
        e_h, g_h = b.energy_grad(flat * scale)
        assert np.array_equal(e_d, e_h)
        assert np.array_equal(g_d, g_h)
        for kind, i, prob in checks[::2]:
            t = flat[b.offsets[i]:b.offsets[i + 1]] * scale
            assert abs(e_d[i] - prob.energy(t)) < TOL_E


def test_device_entry_energy_only_and_argument_checks():
    import torch
    Hs, As, nes, thetas, _ = _mixed()
    b = vq.Batch(Hs[:4], As[:4], nes[:4])
    flat = np.concatenate(thetas[:4])
    th = torch.tensor(flat, dtype=torch.float64, device="cuda")
    e = torch.full((b.S,), float("nan"), dtype=torch.float64, device="cuda")
    b.energy_grad_device(th, e)
    e_h, _ = b.energy_grad(flat, grad=False)
    assert np.array_equal(e.cpu().numpy(), e_h)
    with pytest.raises(ValueError):
        b.energy_grad_device(th[:-1], e)
    with pytest.raises(ValueError):
        b.energy_grad_device(th.float(), e)
    with pytest.raises(ValueError):
        b.energy_grad_device(th.cpu(), e)
