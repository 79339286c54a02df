"""Writes tests/golden/single24.json: the oracle's energy and sixteen
four-term shift-rule gradient components for the 24-qubit, 12-electron
workload (integrals seed 4, theta = uniform_theta(1, M)), the configuration
bench.py times as `single24`.  Components: the first, a middle and the last
single, the first, a middle and the last double, and ten more drawn with a
fixed seed.  Calls only the oracle (CI space, float64); takes about an hour
on an 8-core CPU.

    python tests/golden/make_single24.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import fermion as F  # noqa: E402
from vqe_inputs import random_integrals, uniform_theta  # noqa: E402

N, NE, SEED = 24, 12, 4


def components(M, singles):
    fixed = {0, singles // 2, singles - 1, singles, 900, M - 1}
    rng = np.random.default_rng(2424)
    extra = [int(k) for k in rng.permutation(M) if int(k) not in fixed][:10]
    return sorted(fixed | set(extra))


def main():
    t0 = time.time()
    h0, h, g = random_integrals(N, SEED)
    prob = F.Problem(N, NE, h0, h, g)
    theta = uniform_theta(1, prob.n_params)
    singles = sum(1 for e in F.uccsd_excitations(N, NE) if len(e) == 2)
    comps = components(prob.n_params, singles)
    energy = prob.energy(theta)
    print(f"energy {energy:.12f} ({time.time() - t0:.0f} s)", flush=True)
    grad = []
    for k in comps:
        grad.append(float(prob.grad_shift(theta, [k])[0]))
        print(f"component {k}: {grad[-1]:.15f} ({time.time() - t0:.0f} s)", flush=True)
    out = {"n_qubits": N, "n_electrons": NE, "integrals_seed": SEED, "theta_seed": 1,
           "n_params": int(prob.n_params), "energy": float(energy),
           "grad_components": {str(k): v for k, v in zip(comps, grad)},
           "source": "oracle/fermion.py Problem.energy and Problem.grad_shift (float64)",
           "seconds": round(time.time() - t0, 1)}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "single24.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
