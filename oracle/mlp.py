"""Oracle of the warm-start MLP (test infrastructure only).

A project addition, not part of the paper: an MLP maps a geometry descriptor
x = [lambda, upper triangle of h(lambda)] to UCCSD amplitudes theta (the
converged amplitudes of plain VQE at neighbouring geometries of a bond-stretch
scan, Sec. 3.1 "Results for bond stretching", are its training data).

Network: for layers l = 1..L, z_l = a_{l-1} W_l^T + b_l, a_l = GELU(z_l)
for hidden layers and a_L = z_L; GELU(z) = z/2 (1 + erf(z / sqrt 2)) (exact
form, Hendrycks & Gimpel 2016).  Loss: mean squared error over all outputs.
Optimiser: Adam (Kingma & Ba 2015).

Precision model of the GPU kernels, reproduced here in float64:
* GEMM operands (activations, weights, back-propagated errors) are rounded
  to bfloat16 (round to nearest, ties to even) before each product; the
  products accumulate in float32 on the GPU (float64 here);
* biases, pre-activations, GELU, the loss, master weights and Adam moments
  are float32 on the GPU (float64 here, unrounded).
``rounding=False`` gives the plain float64 network (used for FD pins).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erf


def bf16(x) -> np.ndarray:
    """Round to the nearest bfloat16 (8 significant bits), ties to even,
    computed on float32 bit patterns: values must be float32-representable."""
    a = np.asarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    rounded = (u + 0x7FFF + ((u >> 16) & 1)) >> 16
    out = (rounded << 16).astype(np.uint32).view(np.float32)
    out = np.where(np.isnan(a), a, out)
    return out.astype(np.float64)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def unpack(params, widths):
    """Packed layout: for each layer, W [out][in] row-major then b [out]."""
    out, off = [], 0
    for fi, fo in zip(widths[:-1], widths[1:]):
        W = params[off:off + fo * fi].reshape(fo, fi)
        off += fo * fi
        b = params[off:off + fo]
        off += fo
        out.append((W, b))
    assert off == params.size
    return out


def n_params(widths):
    return sum(fo * fi + fo for fi, fo in zip(widths[:-1], widths[1:]))


def forward(params, widths, x, rounding=True):
    """Returns (output, cache) for a batch x [B, in]."""
    r = bf16 if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    layers = unpack(np.asarray(params, dtype=np.float64), widths)
    a = np.asarray(x, dtype=np.float64)
    cache = []
    for li, (W, b) in enumerate(layers):
        a_in = r(a)
        z = a_in @ r(W).T + b
        last = li == len(layers) - 1
        a = z if last else gelu(z)
        cache.append((a_in, z))
    return a, cache


def loss_and_grad(params, widths, x, y, rounding=True):
    """MSE loss and its gradient with respect to the packed parameters."""
    r = bf16 if rounding else (lambda v: np.asarray(v, dtype=np.float64))
    layers = unpack(np.asarray(params, dtype=np.float64), widths)
    out, cache = forward(params, widths, x, rounding)
    diff = out - y
    loss = float(np.mean(diff * diff))
    dz = 2.0 * diff / diff.size
    grads = []
    for li in range(len(layers) - 1, -1, -1):
        W, _ = layers[li]
        a_in, z = cache[li]
        if li != len(layers) - 1:
            dz = dz * gelu_grad(z)
        dzr = r(dz)
        dW = dzr.T @ a_in
        db = dz.sum(axis=0)
        grads.append((dW, db))
        if li > 0:
            dz = dzr @ r(W)
    grads.reverse()
    flat = np.concatenate([np.concatenate([dW.ravel(), db]) for dW, db in grads])
    return loss, flat


def adam_step(params, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t (1-based); returns new (params, m, v)."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return params - lr * mh / (np.sqrt(vh) + eps), m, v


def init_params(widths, seed):
    """He-normal weights, zero biases (float32-representable values)."""
    rng = np.random.default_rng(seed)
    parts = []
    for fi, fo in zip(widths[:-1], widths[1:]):
        parts.append(rng.normal(0.0, math.sqrt(2.0 / fi), size=fo * fi))
        parts.append(np.zeros(fo))
    return np.concatenate(parts).astype(np.float32).astype(np.float64)
