"""Writes tests/golden/long22.json: the oracle's energy and eight four-term
shift-rule gradient components for a 22-qubit, 10-electron UCCSD problem
(integrals seed 2201, theta = uniform_theta(2202, M)).  Its 462 beta strings
per alpha string are more than one wave's rows hold, the case where the
string-product H-apply spreads a row over several waves.  Components: the
first and the last single, the first and the last double, and four more drawn
with a fixed seed.  Calls only the oracle (CI space, float64); takes a few
minutes on a CPU.

    python tests/golden/make_long22.py
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

N, NE, SEED, THETA_SEED = 22, 10, 2201, 2202


def main():
    t0 = time.time()
    prob = F.Problem(N, NE, *random_integrals(N, SEED))
    theta = uniform_theta(THETA_SEED, prob.n_params)
    M = prob.n_params
    singles = sum(1 for e in F.uccsd_excitations(N, NE) if len(e) == 2)
    fixed = {0, singles - 1, singles, M - 1}
    rng = np.random.default_rng(2222)
    extra = [int(k) for k in rng.permutation(M) if int(k) not in fixed][:4]
    comps = sorted(fixed | set(extra))
    energy = prob.energy(theta)
    grad = prob.grad_shift(theta, comps)
    out = {"n_qubits": N, "n_electrons": NE, "integrals_seed": SEED, "theta_seed": THETA_SEED,
           "n_params": int(M), "energy": float(energy),
           "grad_components": {str(k): float(v) for k, v in zip(comps, np.asarray(grad))},
           "source": "oracle/fermion.py Problem.energy and Problem.grad_shift (float64)",
           "seconds": round(time.time() - t0, 1)}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "long22.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
