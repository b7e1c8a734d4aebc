"""Training loss, its gradient by finite differences, and Adam (oracle; test infrastructure).

Paper passages followed:
  * Section III-A: networks are trained with a cross-entropy loss whose
    value in bits per pixel indicates the rate without header.
  * Section IV: the network can be retrained on domain data (MRI).

Readings where the paper is silent: the loss is the mean over sampled pixels of
-log2 P(target | window) under the discretised logistic mixture; windows
are taken inside each slice with the same dummy rule as coding; the
optimiser is Adam (Kingma and Ba, 2015) with lr 1e-3, betas (0.9, 0.999),
eps 1e-8.

Parity (CPU tests in tests/test_oracle_nll.py):
  * sample_features: equal, pixel by pixel, to the whole-slice window
    matrix (itself pinned by hand-derived golden windows) and to the
    one-pixel window reader;
  * nll_bits: equal to a per-sample loop over CDF differences (not the log
    form the loss uses);
  * nll_and_grad_fd: equal to hand-derived derivatives of a single
    logistic (five identical components, weights zero), to the chain rule
    through the last layer, and to the softmax shift invariance;
  * adam_update: equal to torch.optim.Adam over five steps.
"""
from __future__ import annotations

import math

import numpy as np

from .mixture import log_pmf
from .network import mlp_forward, mixture_head
from .window import NEIGHBOURS, scale

PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def sample_features(stack, idx) -> np.ndarray:
    """Windows of sampled pixels (slice, y, x) taken inside their slice, (n, 12) FP64."""
    stack = np.asarray(stack)
    idx = np.asarray(idx, dtype=np.int64)
    _, h, w = stack.shape
    s, y, x = idx[:, 0], idx[:, 1], idx[:, 2]
    out = np.zeros((idx.shape[0], len(NEIGHBOURS)), dtype=np.float64)
    for k, (dy, dx) in enumerate(NEIGHBOURS):
        yy, xx = y + dy, x + dx
        ok = (yy >= 0) & (yy < h) & (xx >= 0) & (xx < w)
        out[ok, k] = scale(stack[s[ok], yy[ok], xx[ok]])
    return out


def nll_bits(weights, stack, idx) -> float:
    """Mean -log2 P(target) over the sampled pixels, FP64."""
    feats = sample_features(stack, idx)
    target = np.asarray(stack)[idx[:, 0], idx[:, 1], idx[:, 2]].astype(np.int64)
    o = mlp_forward(feats, *(weights[k] for k in PARAM_ORDER))
    pi, mu, inv_s = mixture_head(o)
    lp = log_pmf(target, pi, mu, inv_s)
    return float(-np.mean(lp) / math.log(2.0))


def nll_and_grad_fd(weights, stack, idx, picks, h: float = 1e-6):
    """Loss and central-difference derivatives d loss / d param for picked entries.

    picks: list of (name, flat_index).  Parameters are perturbed in FP64.
    """
    base = {k: np.asarray(weights[k], dtype=np.float64).copy() for k in PARAM_ORDER}
    loss = nll_bits(base, stack, idx)
    grads = []
    for name, i in picks:
        p = base[name].reshape(-1)
        keep = p[i]
        p[i] = keep + h
        lp = nll_bits(base, stack, idx)
        p[i] = keep - h
        lm = nll_bits(base, stack, idx)
        p[i] = keep
        grads.append((lp - lm) / (2.0 * h))
    return loss, np.asarray(grads)


def adam_update(p, g, m, v, step: int, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (bias-corrected moments), FP64; returns (p, m, v)."""
    p = np.asarray(p, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    m = b1 * np.asarray(m, dtype=np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, dtype=np.float64) + (1.0 - b2) * g * g
    mhat = m / (1.0 - b1 ** step)
    vhat = v / (1.0 - b2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v
