"""Writes tests/golden/single24.json: the oracle's energy and four-term
shift-rule gradient components for the 24-qubit, 12-electron workload
(integrals seed 4, theta = uniform_theta(1, M)), the configuration bench.py
times as `single24`.  Calls only the oracle (CI space, float64); takes
several minutes on a CPU.

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
COMPONENTS = [0, 71, 900, 1817]   # first single, last single, a double, the last double


def main():
    t0 = time.time()
    h0, h, g = random_integrals(N, SEED)
    prob = F.Problem(N, NE, h0, h, g)
    theta = uniform_theta(1, prob.n_params)
    energy = prob.energy(theta)
    grad = prob.grad_shift(theta, COMPONENTS)
    out = {"n_qubits": N, "n_electrons": NE, "integrals_seed": SEED, "theta_seed": 1,
           "n_params": int(prob.n_params), "energy": float(energy),
           "grad_components": {str(k): float(v) for k, v in zip(COMPONENTS, np.asarray(grad))},
           "source": "oracle/fermion.py Problem.energy and Problem.grad_shift (float64)",
           "seconds": round(time.time() - t0, 1)}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "single24.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
