"""Discretised logistic mixture over 256 grey levels (oracle; test infrastructure).

Paper passages followed:
  * Equation (1): each pixel is coded with P(x_i | x_j .. x_k), a PDF over
    its possible values given the window.
  * Section I: PixelCNN++ parametrises a mixture of logistics; Section IV-C
    (Higher Bit Depth) names the discretised mixture of logistics.
  * Section III-A: the validation loss in bits per pixel measures the rate
    excluding header information.

Readings where the paper is silent: level v owns the interval [beta_v, beta_{v+1}) with
beta_v = (2v - 1)/255 - 1 for v = 1..255, beta_0 = -inf, beta_256 = +inf,
so the two end bins are open and the 256 masses sum to one exactly.

Parity: pinned by the telescoping sum, the single-logistic closed form
P(v) = tanh(inv_s/510) for a bin-centred mean, mirror symmetry for zero
means, and brute-force ideal code length.
"""
from __future__ import annotations

import math

import numpy as np

N_LEVELS = 256


def bin_edges() -> np.ndarray:
    """Interior bin edges beta_1..beta_255 in FP64 (index 0 is beta_1)."""
    v = np.arange(1, N_LEVELS, dtype=np.float64)
    return (2.0 * v - 1.0) / 255.0 - 1.0


def sigmoid(t):
    """Logistic function 1/(1+exp(-t)) in FP64, evaluated without overflow."""
    t = np.asarray(t, dtype=np.float64)
    out = np.empty_like(t)
    pos = t >= 0
    out[pos] = 1.0 / (1.0 + np.exp(-t[pos]))
    e = np.exp(t[~pos])
    out[~pos] = e / (1.0 + e)
    return out


def mixture_cdf(beta, pi, mu, inv_s):
    """C(beta) = sum_k pi_k sigma((beta - mu_k) inv_s_k); beta broadcasts against (..., 5)."""
    b = np.asarray(beta, dtype=np.float64)[..., None]
    return np.sum(pi * sigmoid((b - mu) * inv_s), axis=-1)


def _softplus(t):
    t = np.asarray(t, dtype=np.float64)
    return np.maximum(t, 0.0) + np.log1p(np.exp(-np.abs(t)))


def log_pmf(v, pi, mu, inv_s):
    """Natural log of P(v) for levels v (int array broadcasting with params (..., 5)).

    Per component, with A = (beta_{v+1} - mu) inv_s and B = (beta_v - mu) inv_s:
      interior: log(sigma(A) - sigma(B)) = -softplus(-A) - softplus(B) + log(-expm1(B - A))
      v = 0:    log sigma(A)
      v = 255:  -softplus(B)
    combined over components with log-sum-exp of log pi_k.
    """
    v = np.asarray(v, dtype=np.int64)
    vv = v[..., None]
    hi = (2.0 * (vv + 1) - 1.0) / 255.0 - 1.0
    lo = (2.0 * vv - 1.0) / 255.0 - 1.0
    A = (hi - mu) * inv_s
    B = (lo - mu) * inv_s
    with np.errstate(divide="ignore", invalid="ignore"):
        interior = -_softplus(-A) - _softplus(B) + np.log(-np.expm1(B - A))
    lp = np.where(vv == 0, -_softplus(-A), np.where(vv == N_LEVELS - 1, -_softplus(B), interior))
    with np.errstate(divide="ignore"):
        terms = np.log(pi) + lp
    m = terms.max(axis=-1, keepdims=True)
    return (m + np.log(np.sum(np.exp(terms - m), axis=-1, keepdims=True)))[..., 0]


def pmf_table(pi, mu, inv_s) -> np.ndarray:
    """All 256 masses of one pixel by CDF differences, FP64 (for pins only)."""
    e = bin_edges()
    c = np.concatenate([[0.0], mixture_cdf(e, pi, mu, inv_s), [1.0]])
    return np.diff(c)


def ideal_bits(v, pi, mu, inv_s) -> float:
    """Ideal code length -sum log2 P(v) over all given pixels (math.fsum)."""
    lp = log_pmf(v, pi, mu, inv_s)
    return math.fsum((-lp / math.log(2.0)).ravel().tolist())


def ideal_bits_image(img, weights) -> float:
    """Ideal code length of a whole image under the network (bits)."""
    from .window import causal_features
    from .network import mlp_forward, mixture_head
    o = mlp_forward(causal_features(img), weights["W1"], weights["b1"], weights["W2"],
                    weights["b2"], weights["W3"], weights["b3"])
    pi, mu, inv_s = mixture_head(o)
    return ideal_bits(np.asarray(img).ravel(), pi, mu, inv_s)
