"""Density network and mixture head (oracle; test infrastructure).

Paper passages followed:
  * Section II-A: a neural network maps the neighbourhood window of a pixel
    to a PDF over all pixel values.
  * Section II-B (Preprocessor): with wavefront parallelism the network
    takes a matrix, one row per pixel window.
  * Section II-B (Neural Network Architecture): a dense network; the
    workloads here use 12 -> H -> H -> 15 with ReLU (two hidden layers).
  * Section I and Section IV-B/IV-C (Higher Bit Depth): the alternative
    output is a (discretised) mixture of logistics as in PixelCNN++.

Readings where the paper is silent: outputs are ordered [5 mixture logits, 5 means,
5 log-scales]; means live in the scaled [-1, 1] domain; log-scales are
clamped below at -7; inverse scale = exp(-log_scale).

Parity: pinned by the zero-weight identity, a hand example, and the
PyTorch FP64 linear/ReLU chain (library routine).
"""
from __future__ import annotations

import numpy as np

N_MIX = 5
N_OUT = 3 * N_MIX
LOG_SCALE_MIN = -7.0


def mlp_forward(feats, W1, b1, W2, b2, W3, b3) -> np.ndarray:
    """o = W3 relu(W2 relu(W1 f + b1) + b2) + b3 for each row f, in FP64.

    feats: (n, k_in); W*: [out, in]; returns (n, n_out) FP64.
    """
    f = np.asarray(feats, dtype=np.float64)
    w1, w2, w3 = (np.asarray(a, dtype=np.float64) for a in (W1, W2, W3))
    c1, c2, c3 = (np.asarray(a, dtype=np.float64) for a in (b1, b2, b3))
    h1 = np.maximum(f @ w1.T + c1, 0.0)
    h2 = np.maximum(h1 @ w2.T + c2, 0.0)
    return h2 @ w3.T + c3


def mixture_head(o):
    """Mixture parameters from network outputs, FP64.

    Returns (pi, mu, inv_s), each (..., 5): pi = softmax(logits),
    mu = means, inv_s = exp(-max(log_scale, -7)).
    """
    o = np.asarray(o, dtype=np.float64)
    logits = o[..., 0:N_MIX]
    mu = o[..., N_MIX:2 * N_MIX]
    log_s = np.maximum(o[..., 2 * N_MIX:3 * N_MIX], LOG_SCALE_MIN)
    z = logits - logits.max(axis=-1, keepdims=True)
    e = np.exp(z)
    pi = e / e.sum(axis=-1, keepdims=True)
    return pi, mu.copy(), np.exp(-log_s)
