"""Pins of the reduced-precision oracle (BF16 / FP8 e4m3 network forms)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import lowp


def test_round_bf16_matches_torch_and_ties():
    rng = np.random.default_rng(5)
    x = np.concatenate([
        rng.standard_normal(50000).astype(np.float32),
        (rng.standard_normal(20000) * 1e-30).astype(np.float32),
        (rng.standard_normal(20000) * 1e20).astype(np.float32),
        # exact ties: low half 0x8000 with both parities of the kept half
        (np.arange(1000, dtype=np.uint32) << 16 | 0x8000).view(np.float32),
    ])
    want = torch.from_numpy(x).to(torch.bfloat16).to(torch.float32).numpy()
    np.testing.assert_array_equal(lowp.round_bf16(x), want)
    # 1 + 2^-8 is halfway between 1 and 1 + 2^-7: ties to even gives 1
    assert lowp.round_bf16(np.float32(1 + 2 ** -8)) == 1.0
    # 1 + 3 * 2^-8 is halfway between 1 + 2^-7 (odd) and 1 + 2^-6 (even)
    assert lowp.round_bf16(np.float32(1 + 3 * 2 ** -8)) == np.float32(1 + 2 ** -6)
    assert lowp.bf16_bits(np.float32(-2.0)) == 0xC000


def test_e4m3_code_table_matches_torch():
    codes = np.arange(256, dtype=np.uint8)
    want = torch.from_numpy(codes).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    got = lowp.e4m3_value(codes)
    np.testing.assert_array_equal(np.isnan(got), np.isnan(want))
    ok = ~np.isnan(want)
    np.testing.assert_array_equal(got[ok], want[ok])
    # hand values: largest finite, smallest subnormal, smallest normal, one
    assert lowp.e4m3_value(0x7E) == 448.0
    assert lowp.e4m3_value(0x01) == 2.0 ** -9
    assert lowp.e4m3_value(0x08) == 2.0 ** -6
    assert lowp.e4m3_value(0x38) == 1.0
    assert lowp.e4m3_value(0xB8) == -1.0


def test_e4m3_encode_matches_torch_in_range():
    rng = np.random.default_rng(6)
    codes = np.arange(0x7F)
    vals = lowp.e4m3_value(codes)
    mids = (vals[1:] + vals[:-1]) / 2  # exact ties between neighbouring codes
    x = np.concatenate([
        rng.uniform(-448, 448, 40000),
        rng.standard_normal(40000) * 0.01,
        mids, -mids, vals, -vals, [0.0, 447.9, 448.0, -448.0],
    ]).astype(np.float32)
    want = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    got = lowp.e4m3_encode(x)
    # torch keeps the sign of zero; this format writes every zero as +0
    want = np.where(want == 0x80, 0, want)
    np.testing.assert_array_equal(got, want)
    # saturation above the largest finite value
    assert lowp.e4m3_encode(np.float32(460.0)) == 0x7E
    assert lowp.e4m3_encode(np.float32(-1e6)) == 0xFE
    # ties to even by hand: 1.5 * 2^-9 between codes 1 and 2 -> 2; 2^-10 -> 0
    assert lowp.e4m3_encode(np.float32(1.5 * 2 ** -9)) == 2
    assert lowp.e4m3_encode(np.float32(2 ** -10)) == 0


def test_fp8_scale_rule():
    w = np.array([[0.5, -3.5, 1e-3], [2.0, 0.0, -0.25]], dtype=np.float32)
    codes, scale = lowp.quantize_matrix(w, "fp8")
    assert scale == np.float32(np.float32(3.5) / np.float32(448.0))
    assert codes[0, 1] == 0xFE  # the largest magnitude maps to -448
    assert codes[1, 1] == 0
    back = lowp.e4m3_value(codes) * float(scale)
    assert np.all(np.abs(back - w) <= np.abs(w) * 2 ** -4 + float(scale) * 2 ** -10)
    # an all-zero matrix keeps scale 1
    assert lowp.quantize_matrix(np.zeros((2, 2), np.float32), "fp8")[1] == 1.0


def _exact_model(h):
    """Weights that BF16 and e4m3 with scale 2^-8 store exactly: element
    [0][0] = 1.75 (so max|W| / 448 = 2^-8) alone in its row, every other row
    with two entries from {+-0.5, +-0.25}; biases in {-1, 0, 1}."""
    rng = np.random.default_rng(7)

    def mat(o, i):
        m = np.zeros((o, i), np.float32)
        m[0, 0] = 1.75
        for r in range(1, o):
            cols = rng.choice(i, 2, replace=False)
            m[r, cols] = rng.choice([-0.5, -0.25, 0.25, 0.5], 2)
        return m

    def bias(n):
        return rng.integers(-1, 2, n).astype(np.float32)

    return {"W1": mat(h, 12), "b1": bias(h), "W2": mat(h, h), "b2": bias(h),
            "W3": mat(15, h), "b3": bias(15)}


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_lowp_forward_equals_fp64_when_roundings_are_exact(dtype):
    # sparse power-of-two weights, integer biases, inputs in {-1, 0, 1} (grey
    # levels 0 and 255, dummy 0): every hidden activation is a multiple of
    # 2^-4 below 8, exact in BF16, so both forms must agree exactly; a dropped
    # term, misplaced scale or transposed operand does not survive this.
    w = _exact_model(16)
    img = np.where(np.random.default_rng(8).random((6, 7)) < 0.5, 0, 255).astype(np.uint8)
    f = oracle.causal_features(img).reshape(-1, 12)
    qm = lowp.quantize_weights(w, dtype)
    if dtype == "fp8":
        np.testing.assert_array_equal(qm["scales"], np.float32(2.0 ** -8))
    eff = lowp.effective_weights(qm)
    for k in ("W1", "W2", "W3"):
        np.testing.assert_array_equal(eff[k], w[k].astype(np.float64))
    h1 = np.maximum(f @ eff["W1"].T + eff["b1"], 0)
    h2 = np.maximum(h1 @ eff["W2"].T + eff["b2"], 0)
    assert np.array_equal(lowp.round_bf16(h1.astype(np.float32)), h1)
    assert np.array_equal(lowp.round_bf16(h2.astype(np.float32)), h2)
    want = oracle.mlp_forward(f, w["W1"], w["b1"], w["W2"], w["b2"], w["W3"], w["b3"])
    np.testing.assert_array_equal(lowp.mlp_forward_lowp(f, qm), want)


def test_lowp_forward_rounds_hidden_activations():
    # one pixel, h = 16: hidden unit 0 gets z = 1 + 2^-8 (exact in FP64), which
    # BF16 rounds to 1 (tie to even); output 0 copies it through layer 2.
    h = 16
    w = {k: np.zeros(s, np.float32) for k, s in
         (("W1", (h, 12)), ("b1", h), ("W2", (h, h)), ("b2", h), ("W3", (15, h)), ("b3", 15))}
    w["W1"][0, 11] = 1.0
    w["b1"][0] = 2.0 ** -8
    w["W2"][0, 0] = 1.0
    w["W3"][0, 0] = 1.0
    f = np.zeros((1, 12))
    f[0, 11] = 1.0
    qm = lowp.quantize_weights(w, "bf16")
    assert lowp.mlp_forward_lowp(f, qm)[0, 0] == 1.0
    assert oracle.mlp_forward(f, *(w[k] for k in ("W1", "b1", "W2", "b2", "W3", "b3")))[0, 0] \
        == 1.0 + 2.0 ** -8
    # inputs are rounded too: feature 1 + 2^-8 counts as 1
    f2 = f.copy()
    f2[0, 11] = 1.0 + 2.0 ** -8
    w["b1"][0] = 0.0
    qm = lowp.quantize_weights(w, "bf16")
    assert lowp.mlp_forward_lowp(f2, qm)[0, 0] == 1.0


def test_w8a8_multiplier_hand_values():
    assert lowp.w8a8_multiplier(1.0) == 256.0      # 256 <= 448 < 512
    assert lowp.w8a8_multiplier(448.0) == 1.0
    assert lowp.w8a8_multiplier(449.0) == 0.5
    assert lowp.w8a8_multiplier(0.001) == 2.0 ** 18  # 262.1 <= 448 < 524.3
    assert lowp.w8a8_multiplier(0.0) == 1.0


def test_w8a8_forward_equals_fp64_when_roundings_are_exact():
    # one nonzero per row from {+-1, +-0.5} (plus the 1.75 that fixes the
    # weight scale at 2^-8, on a unit that is always 0 after ReLU), biases in
    # {0, 1}: every layer input has at most 3 significant bits, so its e4m3
    # rounding after the power-of-two multiplier is exact and the W8A8 form
    # must equal the FP64 network; a wrong multiplier or a scale applied the
    # wrong way round does not survive this.
    rng = np.random.default_rng(9)
    h = 16

    def mat(o, i):
        m = np.zeros((o, i), np.float32)
        m[0, 0] = 1.75
        for r in range(1, o):
            m[r, rng.integers(1, i)] = rng.choice([-1.0, -0.5, 0.5, 1.0])
        return m

    w = {"W1": mat(h, 12), "W2": mat(h, h), "W3": mat(15, h),
         "b1": rng.integers(0, 2, h).astype(np.float32), "b2": rng.integers(0, 2, h).astype(np.float32),
         "b3": rng.integers(-1, 2, 15).astype(np.float32)}
    w["b1"][0] = -1.75  # unit 0 of layer 1 is 0 for every input in {-1, 0, 1}
    img = np.where(np.random.default_rng(10).random((7, 9)) < 0.5, 0, 255).astype(np.uint8)
    f = oracle.causal_features(img).reshape(-1, 12)
    keys = ("W1", "b1", "W2", "b2", "W3", "b3")
    h1 = np.maximum(f @ w["W1"].T.astype(np.float64) + w["b1"], 0)
    h2 = np.maximum(h1 @ w["W2"].T.astype(np.float64) + w["b2"], 0)
    qm = lowp.quantize_weights(w, "fp8a8", act_max=(1.0, h1.max(), h2.max()))
    np.testing.assert_array_equal(qm["scales"], np.float32(2.0 ** -8))
    assert qm["mults"][0] == 256.0
    want = oracle.mlp_forward(f, *(w[k] for k in keys))
    np.testing.assert_array_equal(lowp.mlp_forward_lowp(f, qm), want)


def test_w8a8_forward_rounds_inputs_to_e4m3():
    # a single path: output 0 = feature 11 * 1; the feature -1 + 2/255 (grey
    # level 1) times 256 is -253.99.., whose nearest e4m3 value is -256
    h = 16
    w = {k: np.zeros(s, np.float32) for k, s in
         (("W1", (h, 12)), ("b1", h), ("W2", (h, h)), ("b2", h), ("W3", (15, h)), ("b3", 15))}
    w["W1"][1, 11] = -1.0
    w["W2"][1, 1] = 1.0
    w["W3"][0, 1] = 1.0
    f = np.zeros((1, 12))
    f[0, 11] = oracle.scale(1)
    qm = lowp.quantize_weights(w, "fp8a8", act_max=(1.0, 1.0, 1.0))
    # (the weight scales 1/448 are not dyadic: products of them stay within
    # FP32 rounding of 1; without the input rounding the output would be 0.992)
    assert abs(lowp.mlp_forward_lowp(f, qm)[0, 0] - 1.0) < 1e-6
