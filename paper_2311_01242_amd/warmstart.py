"""Learned warm start for VQE along a bond-stretch scan.

The paper runs standard VQE from the Hartree-Fock point at every geometry of
a bond-stretch scan (Sec. 3.1 "Results for bond stretching").  This module
adds, on top of the unchanged method:

1. plain VQE (BFGS from theta = 0, the HF state of Eq. 1) at every scan
   point, through the library's energy + adjoint gradient;
2. an MLP, trained by the library's GPU kernels on the training points'
   (features, converged theta) pairs, that predicts theta at held-out points;
3. VQE from the predicted theta (falling back to theta = 0 when the
   prediction's energy is above the HF energy or not finite), compared with
   plain VQE by the number of BFGS iterations (and energy evaluations) each
   needs to come within 1 mHa of a reference energy: the lower of the two
   runs' final energies (a run that settles in a higher minimum never gets
   there), and, as a second figure, the plain run's own final energy.

Both runs use the same convergence test (max |dE/dtheta| <= gtol) and an
iteration cap well above what the runs need; a point where either run stops
at the cap is excluded from the iteration statistics and counted, and only
converged plain runs are used as training targets.

Split: scan index i is held out when i % 5 == 2 (every fifth point, so the
held-out geometries are interpolations).
"""
from __future__ import annotations

import time

import numpy as np

from . import Ansatz, Hamiltonian, energy_grad, run_vqe
from .mlp import MLP, features

MHA = 1e-3


def iters_to_target(trace, target):
    """First iteration k with E_k <= target (0 if the start qualifies), or
    None if the run never gets there."""
    ok = np.nonzero(np.asarray(trace) <= target)[0]
    return int(ok[0]) if ok.size else None


def run_scan(family, n, ne, lambdas, gtol=1e-6, max_iter=5000, log=None):
    """Plain VQE from theta = 0 at every lambda.  Returns a list of dicts."""
    A = Ansatz.uccsd(n, ne)
    out = []
    for i, lam in enumerate(lambdas):
        h0, h, g = family(lam)
        H = Hamiltonian.from_integrals(n, h0, h, g)
        t0 = time.perf_counter()
        theta, res, trace = run_vqe(H, A, ne, None, max_iter=max_iter, gtol=gtol)
        out.append({"lam": float(lam), "h": h, "theta": theta, "energy": res.energy,
                    "iters": res.iters, "evals": res.n_evals, "converged": res.converged,
                    "trace": trace[:res.iters + 1].copy(), "seconds": time.perf_counter() - t0})
        if log:
            log(f"scan {i} lam={lam:.4f} E={res.energy:.8f} iters={res.iters} converged={res.converged}")
    return A, out


def split(n_points):
    held = [i for i in range(n_points) if i % 5 == 2]
    train = [i for i in range(n_points) if i % 5 != 2]
    return train, held


def train_warmstart(scan, train_idx, hidden=(256, 256), steps=4000, lr=1e-3, seed=0):
    """Train the MLP on (features, theta*) of the training points whose plain
    VQE converged."""
    train_idx = [i for i in train_idx if scan[i]["converged"]]
    X = np.stack([features(scan[i]["lam"], scan[i]["h"]) for i in train_idx])
    Y = np.stack([scan[i]["theta"] for i in train_idx])
    mu, sd = X.mean(axis=0), X.std(axis=0)
    sd[sd == 0] = 1.0
    widths = [X.shape[1], *hidden, Y.shape[1]]
    net = MLP(widths)
    rng = np.random.default_rng(seed)
    parts = []
    for fi, fo in zip(widths[:-1], widths[1:]):
        parts.append(rng.normal(0.0, np.sqrt(2.0 / fi), size=fo * fi))
        parts.append(np.zeros(fo))
    net.set_params(np.concatenate(parts).astype(np.float32))
    loss = net.train((X - mu) / sd, Y, steps, lr=lr)
    return net, (mu, sd), loss


def evaluate(scan, held_idx, net, norm, A, n, ne, family, gtol=1e-6, max_iter=5000):
    """Warm-started VQE at the held-out points against plain VQE."""
    mu, sd = norm
    X = np.stack([features(scan[i]["lam"], scan[i]["h"]) for i in held_idx])
    pred = net.forward((X - mu) / sd).astype(np.float64)
    rows = []
    for k, i in enumerate(held_idx):
        h0, h, g = family(scan[i]["lam"])
        H = Hamiltonian.from_integrals(n, h0, h, g)
        th0 = pred[k]
        e_pred = energy_grad(H, A, ne, th0, grad=False)[0]
        e_hf = energy_grad(H, A, ne, np.zeros(A.n_params), grad=False)[0]
        fallback = (not np.isfinite(e_pred)) or e_pred > e_hf
        if fallback:
            th0 = np.zeros(A.n_params)
        theta, res, trace = run_vqe(H, A, ne, th0, max_iter=max_iter, gtol=gtol)
        trace = trace[:res.iters + 1]
        ref = min(scan[i]["energy"], res.energy)
        target = ref + MHA
        target_plain = scan[i]["energy"] + MHA
        rows.append({
            "lam": scan[i]["lam"], "plain_energy": scan[i]["energy"], "warm_energy": res.energy,
            "ref_energy": ref,
            "plain_iters_to_1mHa": iters_to_target(scan[i]["trace"], target),
            "warm_iters_to_1mHa": iters_to_target(trace, target),
            "plain_iters_to_1mHa_of_plain": iters_to_target(scan[i]["trace"], target_plain),
            "warm_iters_to_1mHa_of_plain": iters_to_target(trace, target_plain),
            "plain_iters": scan[i]["iters"], "warm_iters": res.iters,
            "plain_evals": scan[i]["evals"], "warm_evals": res.n_evals,
            "plain_converged": bool(scan[i]["converged"]), "warm_converged": bool(res.converged),
            "pred_energy": e_pred, "hf_energy": e_hf, "fallback": bool(fallback),
        })
    return rows


def summarize(rows):
    """Statistics over the held-out points where both runs converged (the
    others are counted, not averaged)."""
    both = [r for r in rows if r["plain_converged"] and r["warm_converged"]]

    def stat(key, rs):
        v = np.array([r[key] if r[key] is not None else np.nan for r in rs], float)
        if v.size == 0 or np.all(np.isnan(v)):
            return {"mean": None, "median": None, "missing": int(v.size)}
        return {"mean": float(np.nanmean(v)), "median": float(np.nanmedian(v)),
                "missing": int(np.isnan(v).sum())}
    d = np.array([r["warm_energy"] - r["plain_energy"] for r in both]) if both else np.zeros(0)
    return {
        "points": len(rows),
        "plain_converged": int(sum(r["plain_converged"] for r in rows)),
        "warm_converged": int(sum(r["warm_converged"] for r in rows)),
        "both_converged": len(both),
        "reference": "lower of the plain and warm final energies; iterations to within 1 mHa of it",
        "plain_iters_to_1mHa": stat("plain_iters_to_1mHa", both),
        "warm_iters_to_1mHa": stat("warm_iters_to_1mHa", both),
        "plain_iters_to_1mHa_of_plain": stat("plain_iters_to_1mHa_of_plain", both),
        "warm_iters_to_1mHa_of_plain": stat("warm_iters_to_1mHa_of_plain", both),
        "plain_iters": stat("plain_iters", both), "warm_iters": stat("warm_iters", both),
        "plain_evals": stat("plain_evals", both), "warm_evals": stat("warm_evals", both),
        "fallbacks": int(sum(r["fallback"] for r in rows)),
        "final_energy_diff_max": float(d.max()) if d.size else None,
        "final_energy_diff_min": float(d.min()) if d.size else None,
        "warm_within_1mHa_of_plain": int(np.sum(d <= MHA)),
        "warm_lower_by_over_1mHa": int(np.sum(d < -MHA)),
        "warm_fewer_iters": int(sum(1 for r in both if r["warm_iters_to_1mHa"] is not None and
                                    r["plain_iters_to_1mHa"] is not None and
                                    r["warm_iters_to_1mHa"] < r["plain_iters_to_1mHa"])),
        "warm_reaches_ref": int(sum(1 for r in both if r["warm_iters_to_1mHa"] is not None)),
        "plain_reaches_ref": int(sum(1 for r in both if r["plain_iters_to_1mHa"] is not None)),
    }
