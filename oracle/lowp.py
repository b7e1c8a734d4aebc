"""Reduced-precision forms of the density network (oracle; test infrastructure).

The paper evaluates its network in floating point on the GPU (Section II-B,
Neural Network Architecture) and does not fix a precision.  The reduced-
precision workloads here run the same 12 -> H -> H -> 15 network with BF16
operands and FP32 accumulation, or with FP8 e4m3 weights; this module states
what those forms compute, in FP64 apart from the roundings that define them:

  * BF16: weights, network inputs and hidden activations are rounded to
    BF16 (round to nearest, ties to even) before each product; biases stay
    FP32; z = Wq a + b.
  * FP8 e4m3 weights with one FP32 scale per layer: scale = max|W| / 448 in
    FP32, codes = e4m3(W / scale) (quotient in FP32, round to nearest even,
    saturating at +-448); activations as for BF16; z = scale (Q a) + b.
  * W8A8: those weights, and each layer input rounded to e4m3 after
    multiplying by a power of two m (the largest with max|a| m <= 448 on
    calibration data); z = (scale / m) (Q a_q) + b.

Readings (listed with the others in the design notes): the scale rule, the
order scale-then-bias, and e4m3 as the OCP "FN" variant (no infinities,
largest finite value 448).

Parity: round_bf16 is pinned against PyTorch's CPU bfloat16 conversion and
hand ties; the e4m3 code table and encoder against PyTorch's float8_e4m3fn
and hand values; mlp_forward_lowp against mlp_forward on inputs, weights
and activations that every rounding leaves unchanged (so any dropped term,
wrong scale or transposed operand shows).
"""
from __future__ import annotations

import numpy as np

E4M3_MAX = 448.0


def round_bf16(x) -> np.ndarray:
    """Nearest BF16 value (ties to even) of each FP32 value, as FP32."""
    a = np.ascontiguousarray(x, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lower = u & 0xFFFF
    keep = u >> 16
    up = (lower > 0x8000) | ((lower == 0x8000) & ((keep & 1) == 1))
    keep = keep + up.astype(np.uint64)
    return (keep << 16).astype(np.uint32).view(np.float32).reshape(a.shape)


def bf16_bits(x) -> np.ndarray:
    """uint16 BF16 bit patterns of round_bf16(x)."""
    return (round_bf16(x).view(np.uint32) >> 16).astype(np.uint16)


def e4m3_value(code) -> np.ndarray:
    """Value of each e4m3 code (FP64): sign bit, 4 exponent bits with bias 7,
    3 mantissa bits; exponent 0 is subnormal (m * 2^-9); 0x7F and 0xFF are NaN."""
    c = np.asarray(code, dtype=np.int64)
    sign = np.where(c & 0x80, -1.0, 1.0)
    e = (c >> 3) & 15
    m = c & 7
    mag = np.where(e == 0, m * 2.0 ** -9, (1.0 + m / 8.0) * np.exp2(e - 7.0))
    mag = np.where((c & 0x7F) == 0x7F, np.nan, mag)
    return sign * mag


def _finite_codes():
    codes = np.arange(0x7F, dtype=np.int64)  # non-negative finite codes 0x00..0x7E
    return codes, e4m3_value(codes)


def e4m3_encode(x) -> np.ndarray:
    """e4m3 code nearest to each FP32 value, ties to the even code (mantissa
    bit 0 clear), magnitudes at or above 448 saturated to 448, zero as +0.

    Works by search in the table of the 127 non-negative finite values."""
    a = np.abs(np.asarray(x, dtype=np.float64))
    codes, vals = _finite_codes()
    idx = np.searchsorted(vals, a, side="left")           # vals[idx-1] < a <= vals[idx]
    idx = np.clip(idx, 1, len(vals) - 1)
    lo, hi = vals[idx - 1], vals[idx]
    d_lo, d_hi = a - lo, hi - a
    pick_hi = (d_hi < d_lo) | ((d_hi == d_lo) & (codes[idx] % 2 == 0))
    c = np.where(pick_hi, codes[idx], codes[idx - 1])
    c = np.where(a >= E4M3_MAX, 0x7E, c)
    c = np.where(a == 0.0, 0, c)
    neg = (np.asarray(x, dtype=np.float64) < 0) & (c != 0)
    return (c | np.where(neg, 0x80, 0)).astype(np.uint8)


def quantize_matrix(W, dtype: str):
    """Stored form of one FP32 weight matrix.

    'bf16' -> (uint16 bits, FP32 scale 1.0);  'fp8' -> (uint8 codes, FP32 scale)."""
    w32 = np.asarray(W, dtype=np.float32)
    if dtype == "bf16":
        return bf16_bits(w32), np.float32(1.0)
    if dtype == "fp8":
        amax = np.float32(np.abs(w32).max()) if w32.size else np.float32(0.0)
        scale = np.float32(amax / np.float32(E4M3_MAX)) if amax > 0 else np.float32(1.0)
        q = (w32 / scale).astype(np.float32)  # IEEE FP32 quotient
        return e4m3_encode(q), scale
    raise ValueError(dtype)


def w8a8_multiplier(amax: float) -> np.float32:
    """Power-of-two multiplier 2^k with the largest k such that amax * 2^k <= 448
    (1 for amax <= 0)."""
    if not amax > 0:
        return np.float32(1.0)
    k = 0
    while amax * 2.0 ** k > 448.0:
        k -= 1
    while amax * 2.0 ** (k + 1) <= 448.0:
        k += 1
    return np.float32(2.0 ** k)


def quantize_weights(weights: dict, dtype: str, act_max=None) -> dict:
    """Stored model: {'W1','W2','W3': stored matrices, 'b*': FP32 biases,
    'scales': three FP32 scales, 'dtype': dtype}; for 'fp8a8' also 'mults',
    the activation multipliers of the three layer inputs from their largest
    values act_max (the first is the grey-level range, 1)."""
    out = {"dtype": dtype}
    scales = []
    for k in ("W1", "W2", "W3"):
        stored, s = quantize_matrix(weights[k], "fp8" if dtype == "fp8a8" else dtype)
        out[k] = stored
        scales.append(s)
    for k in ("b1", "b2", "b3"):
        out[k] = np.asarray(weights[k], dtype=np.float32)
    out["scales"] = np.array(scales, dtype=np.float32)
    if dtype == "fp8a8":
        out["mults"] = np.array([w8a8_multiplier(float(a)) for a in act_max], dtype=np.float32)
    return out


def stored_values(qm: dict, key: str) -> np.ndarray:
    """FP64 values of a stored matrix before any scale (BF16 or e4m3 codes)."""
    a = qm[key]
    if qm["dtype"] == "bf16":
        return (a.astype(np.uint32) << 16).view(np.float32).astype(np.float64)
    return e4m3_value(a)


def effective_weights(qm: dict) -> dict:
    """FP64 weights the quantised model stands for (scale times stored value),
    with its FP32 biases; used to evaluate the dtype's network in FP64."""
    out = {}
    for i, k in enumerate(("W1", "W2", "W3")):
        out[k] = stored_values(qm, k) * (float(qm["scales"][i]) if qm["dtype"] != "bf16" else 1.0)
    for k in ("b1", "b2", "b3"):
        out[k] = qm[k].astype(np.float64)
    return out


def mlp_forward_lowp(feats, qm: dict) -> np.ndarray:
    """Network outputs of the reduced-precision form, FP64 apart from the
    roundings of inputs and hidden activations (BF16, or e4m3 after the
    layer's multiplier for 'fp8a8').  feats: (n, 12) FP64 (or FP32) scaled
    window values; returns (n, 15) FP64."""
    if qm["dtype"] == "fp8a8":
        return _forward_w8a8(feats, qm)
    a = round_bf16(np.asarray(feats, dtype=np.float32)).astype(np.float64)
    fp8 = qm["dtype"] == "fp8"
    layers = (("W1", "b1"), ("W2", "b2"), ("W3", "b3"))
    for li, (wk, bk) in enumerate(layers):
        W = stored_values(qm, wk)
        b = qm[bk].astype(np.float64)
        acc = a @ W.T
        z = (float(qm["scales"][li]) * acc if fp8 else acc) + b
        if li == 2:
            return z
        a = round_bf16(np.maximum(z, 0.0).astype(np.float32)).astype(np.float64)
    raise AssertionError


def _forward_w8a8(feats, qm: dict) -> np.ndarray:
    """W8A8: layer input a -> e4m3(RN32(a) * m) (m a power of two, so the
    product is exact), z = (s / m) (Q a_q) + b with FP32 s / m (exact)."""
    a = np.asarray(feats, dtype=np.float32).astype(np.float64)
    for li, (wk, bk) in enumerate((("W1", "b1"), ("W2", "b2"), ("W3", "b3"))):
        m = float(qm["mults"][li])
        aq = e4m3_value(e4m3_encode((a.astype(np.float32) * np.float32(m)).astype(np.float32)))
        W = stored_values(qm, wk)
        d = float(np.float32(qm["scales"][li]) / np.float32(m))
        z = d * (aq @ W.T) + qm[bk].astype(np.float64)
        if li == 2:
            return z
        a = np.maximum(z, 0.0)
    raise AssertionError


def stored_fingerprint(qm: dict) -> int:
    """Model fingerprint of a stored model: FNV-1a 64 over the bytes of W1,
    b1, W2, b2, W3, b3 as stored, then the three scales for FP8."""
    from .container import fingerprint
    arrays = [qm[k] for k in ("W1", "b1", "W2", "b2", "W3", "b3")]
    if qm["dtype"] == "fp8":
        arrays.append(qm["scales"])
    if qm["dtype"] == "fp8a8":
        arrays.append(np.concatenate([qm["scales"], qm["mults"]]).astype(np.float32))
    return fingerprint(arrays)
