"""Autotuner for the launch parameters of the batched path.

For every qubit count of a batch it times (HIP events, via the library's
``vqe_batch_profile``) one evaluation of a sub-batch of that size class under
candidate parameters and keeps the fastest:

* forward run tile budget (LDS bytes per workgroup),
* reverse run tile budget (phi + lambda tiles),
* low-bit tile L of the sector H-apply,
* on the packed layout, the largest run tile (window grouping of the runs).

The three phases are timed separately, so the search is per phase rather
than over the product of the candidate sets.  On the packed sector layout
(UCCSD programs, the default) L is also the layout's block size and the run
budgets play no part: (L, largest run tile) pairs are searched by the time of
the whole evaluation, with the run threads of each pass chosen per pair.  Only tiling changes: the gate order, and therefore the result
up to summation order, never does.  Results are cached in a JSON file keyed
by (device name, layout, qubits, electrons, states).
"""
from __future__ import annotations

import json
import os

import numpy as np

from . import Batch, VQEError, real_enabled, set_run_threads, set_tile_cap, set_tuning

RUN_THREADS = (64, 256, 512, 1024)
# largest packed run tile (entries per vector); 0 = the default (2400, or two of the
# layout's largest blocks when they hold more)
TILE_CAPS = (0, 1200, 1600, 2400)
# with real amplitudes a tile takes half the LDS: larger tiles are candidates too
TILE_CAPS_REAL = (0, 1600, 2400, 3200)

FWD_CANDIDATES = (16 << 10, 32 << 10, 64 << 10, 128 << 10)
ADJ_CANDIDATES = (32 << 10, 64 << 10, 128 << 10)


def _hx_candidates(n):
    return sorted({min(n, L) for L in (10, 11, 12, 13, 14)})


def _device_name():
    """Architecture and compute-unit count of device 0 (the marketing name
    depends on the kernel driver's device-ID tables and is not stable across tools)."""
    try:
        import torch
        p = torch.cuda.get_device_properties(0)
        return f"{getattr(p, 'gcnArchName', 'gpu').split(':')[0]}x{p.multi_processor_count}"
    except Exception:
        return "unknown"


def tune_class(hams, ansatz, n, ne, theta, reps=2, log=None, packed=True):
    """Best (fwd_budget, adj_budget, L) for one size class (batched launches)."""
    def measure(fwd, adj, L):
        set_tuning(n, True, fwd, adj, L)
        b = Batch(hams, [ansatz] * len(hams), [ne] * len(hams))
        b.profile(theta, reps=1)                     # warm-up
        ms = b.profile(theta, reps=reps)
        b.close()
        return ms
    if packed:
        # every (L, tile cap, threads): the run threads of each pass are chosen
        # per (L, cap), then (L, cap) by the time of the whole evaluation
        best, best_t, best_ms = None, None, None
        real = real_enabled()
        for L in sorted({min(n, max(L, ne)) for L in (10, 11, 12, 13, 14)}):
            for cap in (TILE_CAPS_REAL if real else TILE_CAPS):
                set_tile_cap(n, True, cap)
                rec = {}
                for th in (RUN_THREADS[1:] if real else RUN_THREADS[1:3]):
                    set_run_threads(n, True, th, th)
                    try:
                        rec[th] = measure(64 << 10, 64 << 10, L)
                    except VQEError:   # a tile too large for the pair lists or the LDS
                        pass
                if not rec:
                    continue
                tf = min(rec, key=lambda t: rec[t][0])
                ta = min(rec, key=lambda t: rec[t][2])
                m = [rec[tf][0], min(r[1] for r in rec.values()), rec[ta][2]]
                t = sum(m)
                if log:
                    log(f"n={n} packed L={L} cap={cap}: fwd {m[0]:.3f} ({tf}) + H {m[1]:.3f} + "
                        f"adj {m[2]:.3f} ({ta}) ms")
                if best_t is None or t < best_t:
                    best, best_t, best_ms = (64 << 10, 64 << 10, L, tf, ta, cap), t, m
        set_tuning(n, True, *best[:3])
        set_run_threads(n, True, *best[3:5])
        set_tile_cap(n, True, best[5])
        return best, best_ms
    base = (64 << 10, 64 << 10, min(n, 14))
    best = list(base)
    ms = measure(*base)
    best_ms = [ms[0], ms[1], ms[2]]
    for fwd in FWD_CANDIDATES:
        if fwd == best[0]:
            continue
        m = measure(fwd, best[1], best[2])
        if log:
            log(f"n={n} fwd={fwd >> 10}K: {m[0]:.3f} ms")
        if m[0] < best_ms[0]:
            best[0], best_ms[0] = fwd, m[0]
    for adj in ADJ_CANDIDATES:
        if adj == best[1]:
            continue
        m = measure(best[0], adj, best[2])
        if log:
            log(f"n={n} adj={adj >> 10}K: {m[2]:.3f} ms")
        if m[2] < best_ms[2]:
            best[1], best_ms[2] = adj, m[2]
    for L in _hx_candidates(n):
        if L == best[2]:
            continue
        m = measure(best[0], best[1], L)
        if log:
            log(f"n={n} L={L}: {m[1]:.3f} ms")
        if m[1] < best_ms[1]:
            best[2], best_ms[1] = L, m[1]
    set_tuning(n, True, *best)
    return tuple(best), best_ms


def autotune_batch(hams, ansatzes, n_electrons, theta_all, offsets, cache=None, max_per_class=64,
                   log=None, packed=True, tag=""):
    """Tune every size class of a batch and install the results (set_tuning).
    `tag` names the ansatz family in the cache key (empty for UCCSD).
    Returns {n: (fwd, adj, L)}."""
    cache_data = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            cache_data = json.load(f)
    dev = _device_name()
    classes = {}
    for i, (h, a, ne) in enumerate(zip(hams, ansatzes, n_electrons)):
        n = a.info()[0]
        classes.setdefault((n, ne), []).append(i)
    out = {}
    for (n, ne), idx in sorted(classes.items()):
        layout = ("packed-real" if real_enabled() else "packed-win") if packed else "full"
        key = f"{dev}|{layout}|n={n}|ne={ne}|states={len(idx)}"
        if tag:
            key += f"|{tag}"
        if key in cache_data:
            vals = tuple(cache_data[key])
            set_tuning(n, True, *vals[:3])
            if len(vals) >= 5:
                set_run_threads(n, True, *vals[3:5])
            if len(vals) >= 6:
                set_tile_cap(n, True, vals[5])
            out[n] = vals
            continue
        sub = idx[:max_per_class]
        th = np.concatenate([theta_all[offsets[i]:offsets[i + 1]] for i in sub])
        best, _ = tune_class([hams[i] for i in sub], ansatzes[sub[0]], n, ne, th, log=log,
                             packed=packed)
        out[n] = best
        cache_data[key] = list(best)
    if cache:
        with open(cache, "w") as f:
            json.dump(cache_data, f, indent=1, sort_keys=True)
    return out
