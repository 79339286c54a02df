"""Parity at the benchmark's full sizes, in the launch configuration bench.py
times: the 512-state batch (n ~ U{12..20}) with the autotuned parameters,
checked on sampled states against the oracle computed one by one, and the
24-qubit single-state workload against oracle values stored by
tests/golden/make_single24.py (the 24-qubit oracle takes minutes)."""
import json
import os

import numpy as np
import pytest

import paper_2311_01242_amd as vq
from oracle import fermion as F
from vqe_inputs import batch_spec, random_integrals, uniform_theta

pytestmark = pytest.mark.gpu

TOL_E = 1e-10
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.init()
    yield


def test_batch512_sampled_states_match_oracle():
    from paper_2311_01242_amd import autotune
    spec = batch_spec(512)
    Hs, As, nes, thetas, ans = [], [], [], [], {}
    for i, (n, ne, seed) in enumerate(spec):
        h0, h, g = random_integrals(n, seed)
        Hs.append(vq.Hamiltonian.from_integrals(n, h0, h, g))
        if n not in ans:
            ans[n] = vq.Ansatz.uccsd(n, ne)
        As.append(ans[n])
        nes.append(ne)
        thetas.append(uniform_theta(40000 + i, ans[n].n_params))
    flat = np.concatenate(thetas)
    offs = np.cumsum([0] + [a.n_params for a in As])
    autotune.autotune_batch(Hs, As, nes, flat, offs,
                            cache=os.path.join(ROOT, "paper_2311_01242_amd", "tuning_cache.json"))
    b = vq.Batch(Hs, As, nes)
    e, g = b.energy_grad(flat)
    # one state of the largest, a middle and the smallest qubit count
    picks = {}
    for i, (n, ne, seed) in enumerate(spec):
        if n in (20, 16, 12) and n not in picks:
            picks[n] = i
    for n, i in sorted(picks.items()):
        _, ne, seed = spec[i]
        prob = F.Problem(n, ne, *random_integrals(n, seed))
        assert abs(e[i] - prob.energy(thetas[i])) < TOL_E, (n, i)
        if n == 20:   # two gradient components by the shift rule: a single and a double
            idx = [3, prob.n_params - 5]
            gi = g[offs[i]:offs[i + 1]]
            assert np.abs(gi[idx] - prob.grad_shift(thetas[i], idx)).max() < TOL_E


def test_single24_matches_stored_oracle_values():
    with open(os.path.join(ROOT, "tests", "golden", "single24.json")) as f:
        ref = json.load(f)
    n, ne = ref["n_qubits"], ref["n_electrons"]
    h0, h, g = random_integrals(n, ref["integrals_seed"])
    H = vq.Hamiltonian.from_integrals(n, h0, h, g)
    A = vq.Ansatz.uccsd(n, ne)
    assert A.n_params == ref["n_params"]
    theta = uniform_theta(ref["theta_seed"], A.n_params)
    e, grad = vq.energy_grad(H, A, ne, theta)
    assert abs(e - ref["energy"]) < TOL_E
    for k, v in ref["grad_components"].items():
        assert abs(grad[int(k)] - v) < TOL_E, k
