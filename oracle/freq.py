"""Quantisation of the mixture PDF into integer rANS frequency tables
(oracle; test infrastructure).

Paper passages followed:
  * Section II-B (rANS): the entropy coder en-/decodes symbols from the PDF
    the network produces; on the GPU it uses 32-bit arithmetic.
  * Section II-B (Preprocessor): encoder and decoder must see identical
    floating-point results, so the table rule must be evaluated the same
    way on both sides.

The paper does not state the quantisation.  Our reading:
M = 2^16, M' = M - 256 = 65280, and for the cumulative table
    F(0) = 0, F(256) = M,  F(v) = v + min(M', floor(C(beta_v) * M'))  (v = 1..255)
so every symbol gets frequency f_v = F(v+1) - F(v) >= 1 and the table sums
to M whenever C is non-decreasing.

Two evaluations of C are provided:
  * ``table_exact``: FP64 with the exact logistic (used by the pins).
  * the format rule in FP32 (``table_levels32`` / ``table_full32``), which
    is what a decoder must reproduce bit for bit: the logistic is a
    piecewise-linear table on [-16, 16] with step 2^-7 whose 4097 knots are
    S_j = RN32(sigma(-16 + j/128)) and slopes D_j = S_{j+1} - S_j (exact,
    D_4096 = 0), and every operation is one FP32 multiply or add (no fused
    multiply-add).  Per pixel and component, from the FP32 parameters:
        A_k = inv_s_k * 128            B_k = 2048 - mu_k * A_k
    and per level v:
        u = clamp(beta_v * A_k + B_k, 0, 4096)      (the table coordinate of
                                                     (beta_v - mu_k) inv_s_k)
        j = floor(u);  w = u - j;  sigma_hat = S_j + w * D_j
        C = (pi_0 sh_0 + pi_1 sh_1 + pi_2 sh_2) + (pi_3 sh_3 + pi_4 sh_4)
            (each part summed left to right, sh_k = sigma_hat_k)
        q = min(M', floor(C * 65280))
    u is non-decreasing in beta (A_k > 0) and every rounding is monotone, so
    F is non-decreasing in v for any parameters and every table is valid.
    The oracle takes this integer decision in FP32, the kernel's precision.

Parity: pinned by table validity (sum M, every f >= 1) for random
parameters, the strict bound P*M' < f < P*M' + 2 of the exact rule, knot
values against the exact logistic, and monotonicity sweeps of sigma_hat.
"""
from __future__ import annotations

import math

import numpy as np

from .mixture import bin_edges, mixture_cdf

PROB_BITS = 16
M_TOTAL = 1 << PROB_BITS
M_PRIME = M_TOTAL - 256
N_LEVELS = 256

LUT_T_MIN = -16.0
LUT_STEPS_PER_UNIT = 128
LUT_SEGMENTS = 4096


def table_exact(pi, mu, inv_s) -> np.ndarray:
    """Cumulative table F[0..256] (int64) of one pixel from the exact FP64 CDF."""
    c = mixture_cdf(bin_edges(), pi, mu, inv_s)
    q = np.minimum(M_PRIME, np.floor(c * M_PRIME)).astype(np.int64)
    F = np.empty(N_LEVELS + 1, dtype=np.int64)
    F[0] = 0
    F[1:N_LEVELS] = np.arange(1, N_LEVELS) + q
    F[N_LEVELS] = M_TOTAL
    return F


def sigma_lut32():
    """Knots S (4097 FP32) and slopes D (4097 FP32, last is 0) of the table logistic."""
    S = np.empty(LUT_SEGMENTS + 1, dtype=np.float32)
    for j in range(LUT_SEGMENTS + 1):
        t = LUT_T_MIN + j / LUT_STEPS_PER_UNIT
        if t >= 0:
            s = 1.0 / (1.0 + math.exp(-t))
        else:
            e = math.exp(t)
            s = e / (1.0 + e)
        S[j] = np.float32(s)
    D = np.zeros(LUT_SEGMENTS + 1, dtype=np.float32)
    D[:-1] = S[1:] - S[:-1]
    return S, D


_LUT = None


def _lut():
    global _LUT
    if _LUT is None:
        _LUT = sigma_lut32()
    return _LUT


def sigma_hat32(u) -> np.ndarray:
    """Table logistic at FP32 table coordinates u (clamped to [0, 4096]), in FP32."""
    S, D = _lut()
    u = np.asarray(u, dtype=np.float32)
    u = np.where(u > np.float32(0.0), u, np.float32(0.0))
    u = np.minimum(u, np.float32(4096.0))
    j = u.astype(np.int64)
    w = u - j.astype(np.float32)
    return S[j] + w * D[j]


def table_coords32(mu32, is32):
    """Per-component affine map (A, B) of the table coordinate, FP32."""
    A = np.asarray(is32, dtype=np.float32) * np.float32(128.0)
    B = np.float32(2048.0) - np.asarray(mu32, dtype=np.float32) * A
    return A.astype(np.float32), B.astype(np.float32)


def beta32() -> np.ndarray:
    """FP32 bin edges indexed by level 0..256: RN32((2v - 256)/255), ends at -+inf."""
    v = np.arange(N_LEVELS + 1)
    b = np.float32(2.0) * v.astype(np.float32) - np.float32(256.0)
    b = b / np.float32(255.0)
    b[0] = -np.inf
    b[N_LEVELS] = np.inf
    return b.astype(np.float32)


def scale32() -> np.ndarray:
    """FP32 scaled grey levels RN32((2v - 255)/255), v = 0..255."""
    v = np.arange(N_LEVELS).astype(np.float32)
    return ((np.float32(2.0) * v - np.float32(255.0)) / np.float32(255.0)).astype(np.float32)


def _cdf32(beta, pi32, mu32, is32):
    A, B = table_coords32(mu32, is32)

    def part(ks):
        s = None
        for k in ks:
            u = beta * A[..., k:k + 1] + B[..., k:k + 1]
            term = pi32[..., k:k + 1] * sigma_hat32(u)
            s = term if s is None else s + term
        return s

    return part((0, 1, 2)) + part((3, 4))


def table_levels32(levels, pi32, mu32, is32) -> np.ndarray:
    """F(v) by the FP32 format rule for given levels.

    levels: int array (n, m) with values in 0..256; params: FP32 (n, 5).
    Returns int64 (n, m).
    """
    levels = np.asarray(levels, dtype=np.int64)
    pi32 = np.asarray(pi32, dtype=np.float32)
    mu32 = np.asarray(mu32, dtype=np.float32)
    is32 = np.asarray(is32, dtype=np.float32)
    b = beta32()[np.clip(levels, 1, N_LEVELS - 1)]
    C = _cdf32(b, pi32, mu32, is32)
    q = np.minimum(M_PRIME, np.floor(C * np.float32(M_PRIME)).astype(np.int64))
    F = levels + q
    F = np.where(levels <= 0, 0, F)
    F = np.where(levels >= N_LEVELS, M_TOTAL, F)
    return F


def table_full32(pi32, mu32, is32) -> np.ndarray:
    """Whole cumulative tables F[0..256] by the FP32 rule, (n, 257) int64."""
    pi32 = np.atleast_2d(np.asarray(pi32, dtype=np.float32))
    n = pi32.shape[0]
    lv = np.broadcast_to(np.arange(N_LEVELS + 1), (n, N_LEVELS + 1))
    return table_levels32(lv, pi32, np.atleast_2d(mu32), np.atleast_2d(is32))
