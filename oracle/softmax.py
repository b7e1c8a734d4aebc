"""The paper's own density network: six dense layers and a softmax over the 256
grey levels, or the 4096 levels of 12-bit images (oracle; test infrastructure).

Paper passages followed:
  * Section II-B (Neural Network Architecture): a dense network of six dense
    layers (two optional pooling layers, not used here); the output layer has
    256 neurons, one per 8-bit grey level, with a softmax activation; hidden
    layers of 128 to 4096 neurons.
  * Section II-B (Preprocessor): the same arithmetic on both sides of the
    coder, so that encoder and decoder round identically.
  * Section II-B (rANS): the coder consumes the PDF as a cumulative integer
    table.
  * Section IV-C (Higher Bit Depth): 12-bit MRI samples take 4096 output
    neurons (the mixture head did not converge there).

Readings where the paper is silent (the format's choices):
  * the six layers are 12 -> H -> H -> H -> H -> H -> 256 with ReLU after the
    five hidden layers; inputs are the 12-pixel causal window scaled to
    [-1, 1] as for the mixture network;
  * weights are stored in BF16; layer inputs and hidden activations are
    rounded to BF16 (nearest, ties to even) before each product; biases and
    sums are FP32 on the GPU (FP64 here);
  * table rule, FP32 throughout: m = the largest logit; e_v = RN32(exp(o_v - m));
    S = ((S0 + S1) + S2) + S3 with S_b the sum of e_v over the 64 levels of
    block b (v = 64 b .. 64 b + 63) taken in level order; r = 1 / S (correctly
    rounded); p_v = e_v r; block totals T_b of p in level order, block offsets
    O_0 = 0, O_{b+1} = O_b + T_b; inside a block the running sum L (0 at the
    block's first level, L <- L + p_v after level v); C_v = O_b + L_v;
    F(v) = v + min(M', floor(C_v M')) for v = 1..255, F(0) = 0, F(256) = M.
    C is non-decreasing (every addend is >= 0 and FP32 addition is monotone,
    and O_{b+1} = O_b + T_b >= O_b + L of any level of block b), so every
    frequency F(v + 1) - F(v) is at least 1 and they sum to M;
  * N = 2^d levels for d-bit samples (d = 8 or 12): the output layer has N
    neurons, inputs are scaled by (2v - (N - 1)) / (N - 1), and the rule runs
    over N / 64 blocks of 64 levels (S and the offsets summed left to right)
    with M' = M - N; 12-bit streams set the high nibble of the header's dtype
    byte to d - 8 = 4.  The 16-bit table then reserves N / M = 1/16 of the
    mass for the floor of one count per level: at most -log2(15/16) = 0.093
    bits per pixel above the network's own rate.

Parity: the network against PyTorch FP64 linear layers (library routine) and
the zero-weight identity; the softmax against closed forms (equal logits give
p = 1/256, a dominant logit gives 1); the table rule against closed forms
(equal logits give F(v) = 256 v exactly; one dominant level k gives f_k =
M' + 1 and every other f = 1), against the exact FP64 table (within 2 counts)
and against validity on random and extreme logits; the codec by round trips.
"""
from __future__ import annotations

import numpy as np

from .freq import M_PRIME, M_TOTAL
from .lowp import round_bf16

DEPTH = 6
N_LEVELS = 256
BLOCK = 64


def deep_forward(feats, layers) -> np.ndarray:
    """Logits of the six-layer network in FP64: layers = [(W, b)] * 6, W [out, in];
    ReLU after every layer but the last.  feats: (n, 12); returns (n, 256)."""
    a = np.asarray(feats, dtype=np.float64)
    for i, (W, b) in enumerate(layers):
        a = a @ np.asarray(W, dtype=np.float64).T + np.asarray(b, dtype=np.float64)
        if i + 1 < len(layers):
            a = np.maximum(a, 0.0)
    return a


def deep_forward_bf16(feats, layers) -> np.ndarray:
    """The stored form: weights and every layer input rounded to BF16, products and
    sums exact (FP64), biases FP32.  Returns (n, 256) FP64 logits."""
    a = round_bf16(np.asarray(feats, dtype=np.float32)).astype(np.float64)
    for i, (W, b) in enumerate(layers):
        Wb = round_bf16(np.asarray(W, dtype=np.float32)).astype(np.float64)
        z = a @ Wb.T + np.asarray(b, dtype=np.float32).astype(np.float64)
        if i + 1 == len(layers):
            return z
        a = round_bf16(np.maximum(z, 0.0).astype(np.float32)).astype(np.float64)
    raise AssertionError


def softmax_pmf(logits) -> np.ndarray:
    """P(v) = exp(o_v) / sum_u exp(o_u), FP64, each row summing to 1."""
    o = np.asarray(logits, dtype=np.float64)
    e = np.exp(o - o.max(axis=-1, keepdims=True))
    return e / e.sum(axis=-1, keepdims=True)


def ideal_bits_softmax(logits, v) -> float:
    """Sum over rows of -log2 P(v_row), FP64 (log-sum-exp form)."""
    o = np.asarray(logits, dtype=np.float64)
    m = o.max(axis=-1, keepdims=True)
    lse = m[:, 0] + np.log(np.exp(o - m).sum(axis=-1))
    lp = o[np.arange(o.shape[0]), np.asarray(v, dtype=np.int64)] - lse
    return float(-lp.sum() / np.log(2.0))


def levels_of(depth: int) -> int:
    return 1 << depth


def depth_of_levels(n: int) -> int:
    if n not in (256, 4096):
        raise ValueError("256 or 4096 output levels")
    return 8 if n == 256 else 12


def table_softmax_exact(logits) -> np.ndarray:
    """F(v) = v + min(M', floor(C_v M')) with C from the FP64 PMF, M' = M - N:
    (n, N + 1) int64."""
    p = softmax_pmf(logits)
    N = p.shape[-1]
    mp = M_TOTAL - N
    C = np.concatenate([np.zeros((p.shape[0], 1)), np.cumsum(p, axis=-1)], axis=-1)
    v = np.arange(N + 1)
    F = v + np.minimum(mp, np.floor(C * mp)).astype(np.int64)
    F[:, 0] = 0
    F[:, N] = M_TOTAL
    return F


def table_softmax32(logits32) -> np.ndarray:
    """The format's FP32 table rule (module header) on FP32 logits over N = 256 or
    4096 levels: (n, N + 1) int64.

    Every operation is one FP32 operation in the stated order; the exponential
    is the correctly rounded FP32 value of the exact one (through FP64)."""
    o = np.asarray(logits32, dtype=np.float32)
    n, N = o.shape
    depth_of_levels(N)
    mp = M_TOTAL - N
    m = o.max(axis=-1, keepdims=True)
    d = (o - m).astype(np.float32)                       # one FP32 subtraction
    e = np.exp(d.astype(np.float64)).astype(np.float32)
    S = np.zeros(n, dtype=np.float32)
    for b in range(N // BLOCK):
        sb = np.zeros(n, dtype=np.float32)
        for v in range(BLOCK * b, BLOCK * (b + 1)):
            sb = (sb + e[:, v]).astype(np.float32)
        S = sb if b == 0 else (S + sb).astype(np.float32)
    r = (np.float32(1.0) / S).astype(np.float32)
    p = (e * r[:, None]).astype(np.float32)
    C = np.zeros((n, N + 1), dtype=np.float32)
    off = np.zeros(n, dtype=np.float32)
    for b in range(N // BLOCK):
        run = np.zeros(n, dtype=np.float32)
        for v in range(BLOCK * b, BLOCK * (b + 1)):
            C[:, v] = (off + run).astype(np.float32)
            run = (run + p[:, v]).astype(np.float32)
        off = (off + run).astype(np.float32)
    q = np.floor((C * np.float32(mp)).astype(np.float32)).astype(np.int64)
    F = np.arange(N + 1) + np.minimum(mp, q)
    F[:, 0] = 0
    F[:, N] = M_TOTAL
    return F


# --- codec with the softmax network (same container, rANS and wavefront order as the
# mixture network; the header's mixture count is 0 for this head) ----------------------

def stored_fingerprint(layers) -> int:
    """FNV-1a 64 over the stored bytes: BF16 bits of W_i, FP32 b_i, layer by layer."""
    from .container import fingerprint
    from .lowp import bf16_bits
    arrays = []
    for W, b in layers:
        arrays.append(bf16_bits(np.asarray(W, dtype=np.float32)))
        arrays.append(np.asarray(b, dtype=np.float32))
    return fingerprint(arrays)


def header_dtype(depth: int) -> int:
    """The dtype byte of a softmax-network stream: BF16 (1), the depth above 8 in
    the high nibble."""
    return 1 | ((depth - 8) << 4)


def net_depth(layers) -> int:
    return depth_of_levels(int(np.asarray(layers[-1][0]).shape[0]))


def cf_softmax_image(img, layers, logits32=None):
    """(c, f) of every pixel's value by the FP32 rule, raster order.  logits32: FP32
    logits to apply the rule to (default: the FP32 rounding of the oracle's).  The
    bit depth is the network's: 2^d outputs."""
    from .window import causal_features
    d = net_depth(layers)
    img = np.asarray(img, dtype=np.uint8 if d == 8 else np.uint16)
    if logits32 is None:
        logits32 = deep_forward_bf16(causal_features(img, d).reshape(-1, 12), layers).astype(np.float32)
    F = table_softmax32(logits32)
    v = img.reshape(-1).astype(np.int64)
    rows = np.arange(v.size)
    return F[rows, v], F[rows, v + 1] - F[rows, v]


def encode_image_softmax(img, layers, groups, lanes) -> bytes:
    from .container import assemble, pack_header
    from .rans import canonical_order, rans_encode
    d = net_depth(layers)
    img = np.asarray(img, dtype=np.uint8 if d == 8 else np.uint16)
    h, w = img.shape
    c, f = cf_softmax_image(img, layers)
    streams = []
    for grp in canonical_order(h, w, groups, lanes):
        idx = [y * w + x for (y, x, _) in grp]
        streams.append(rans_encode([(c[i], f[i]) for i in idx], [ln for (_, _, ln) in grp], lanes))
    H = np.asarray(layers[0][0]).shape[0]
    hdr = pack_header(h, w, groups, lanes, dtype=header_dtype(d), h1=H, h2=H, n_mix=0,
                      fp=stored_fingerprint(layers))
    return assemble(hdr, streams)


def decode_image_softmax(buf: bytes, layers) -> np.ndarray:
    from .container import parse_header, split_streams
    from .rans import canonical_order, rans_decode
    from .window import pixel_features
    hdr = parse_header(buf)
    d = net_depth(layers)
    if (hdr["n_mix"] != 0 or hdr["dtype"] != header_dtype(d)
            or hdr["fingerprint"] != stored_fingerprint(layers)):
        raise ValueError("stream was coded with another model")
    h, w, groups, lanes = hdr["h"], hdr["w"], hdr["groups"], hdr["lanes"]
    img = np.zeros((h, w), dtype=np.uint8 if d == 8 else np.uint16)
    for grp, words in zip(canonical_order(h, w, groups, lanes), split_streams(buf, groups)):
        def find(i, slot, grp=grp):
            y, x, _ = grp[i]
            o = deep_forward_bf16(pixel_features(img, y, x, d)[None, :], layers).astype(np.float32)
            F = table_softmax32(o)[0]
            v = int(np.searchsorted(F, slot, side="right")) - 1
            img[y, x] = v
            return v, int(F[v]), int(F[v + 1] - F[v])
        _, ok = rans_decode(words, lanes, [ln for (_, _, ln) in grp], find)
        if not ok:
            raise ValueError("corrupt stream")
    return img
