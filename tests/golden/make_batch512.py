"""Writes tests/golden/batch512.json: the oracle's values for the 512-state
batched workload (n ~ U{12..20}, n_e = floor(n/2), state i's integrals from
seed 30000 + i, theta = uniform_theta(40000 + i, M), UCCSD):

* the energy E(theta) of every one of the 512 states (Eq. 1);
* for the first state of every qubit count, eight four-term shift-rule
  gradient components: the first and the last single, the first and the last
  double, and four more drawn with a fixed seed.

Calls only the oracle (CI space, float64) and the seeded input generators;
takes a few minutes on a CPU.

    python tests/golden/make_batch512.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import fermion as F  # noqa: E402
from vqe_inputs import batch_spec, random_integrals, uniform_theta  # noqa: E402

STATES = 512
THETA_SEED0 = 40000


def components(n, ne, M):
    """Gradient components checked for one state of this qubit count."""
    singles = sum(1 for e in F.uccsd_excitations(n, ne) if len(e) == 2)
    fixed = {0, singles - 1, singles, M - 1}
    rng = np.random.default_rng(1000 + n)
    extra = [int(k) for k in rng.permutation(M) if int(k) not in fixed][:4]
    return sorted(fixed | set(extra))


def main():
    t0 = time.time()
    spec = batch_spec(STATES)
    energies = []
    grads = {}
    for i, (n, ne, seed) in enumerate(spec):
        prob = F.Problem(n, ne, *random_integrals(n, seed))
        theta = uniform_theta(THETA_SEED0 + i, prob.n_params)
        energies.append(float(prob.energy(theta)))
        if n not in grads:
            idx = components(n, ne, prob.n_params)
            g = prob.grad_shift(theta, idx)
            grads[n] = {"state": i, "n_params": int(prob.n_params),
                        "components": {str(k): float(v) for k, v in zip(idx, np.asarray(g))}}
        print(f"state {i} n={n} E={energies[-1]:.12f}", flush=True)
    out = {"states": STATES, "theta_seed0": THETA_SEED0, "energies": energies,
           "gradients": {str(n): grads[n] for n in sorted(grads)},
           "source": "oracle/fermion.py Problem.energy and Problem.grad_shift (float64)",
           "seconds": round(time.time() - t0, 1)}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "batch512.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {path} in {out['seconds']} s")


if __name__ == "__main__":
    main()
