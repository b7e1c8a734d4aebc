"""Pins of the oracle's softmax-256 network and its FP32 table rule (CPU): the network
against PyTorch FP64 linear layers and the zero-weight identity, the softmax against closed
forms, the table rule against closed forms, the exact FP64 table and validity on random and
extreme logits, the ideal code length against a direct sum, and the codec by round trips."""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import softmax as sm


def _layers(H=32, seed=5, bias=0.05):
    layers = synth.xavier_deep(H, seed)
    rng = np.random.default_rng(seed + 1)
    return [(W, rng.normal(0, bias, b.shape).astype(np.float32)) for W, b in layers]


def test_six_layers_shapes():
    layers = synth.xavier_deep(128, 3)
    assert [W.shape for W, _ in layers] == [(128, 12)] + [(128, 128)] * 4 + [(256, 128)]
    n = sum(W.size + b.size for W, b in layers)
    assert n == 12 * 128 + 4 * 128 * 128 + 128 * 256 + 5 * 128 + 256   # about 1e5 parameters


def test_forward_matches_torch_linear_chain():
    layers = _layers()
    rng = np.random.default_rng(0)
    f = rng.uniform(-1, 1, (50, 12))
    x = torch.from_numpy(f)
    for i, (W, b) in enumerate(layers):
        x = torch.nn.functional.linear(x, torch.from_numpy(W.astype(np.float64)),
                                       torch.from_numpy(b.astype(np.float64)))
        if i + 1 < len(layers):
            x = torch.relu(x)
    np.testing.assert_allclose(sm.deep_forward(f, layers), x.numpy(), rtol=1e-12, atol=1e-12)


def test_zero_weights_give_the_last_bias():
    layers = [(np.zeros_like(W), b) for W, b in _layers()]
    f = np.random.default_rng(1).uniform(-1, 1, (7, 12))
    out = sm.deep_forward(f, layers)
    assert np.array_equal(out, np.broadcast_to(layers[-1][1].astype(np.float64), out.shape))
    assert np.array_equal(sm.deep_forward_bf16(f, layers), out)


def test_bf16_form_is_exact_on_bf16_values():
    # weights and inputs already BF16 values, activations too: the BF16 form equals FP64
    layers = _layers()
    layers = [(oracle.lowp.round_bf16(W), b) for W, b in layers]
    f = np.array([[(2 * v - 255) / 255 for v in range(12)]], np.float64)
    f = oracle.lowp.round_bf16(f.astype(np.float32)).astype(np.float64)
    a = sm.deep_forward_bf16(f, layers)
    b = sm.deep_forward(f, layers)
    assert np.abs(a - b).max() < 0.02 * np.abs(b).max()


def test_softmax_closed_forms():
    assert np.allclose(sm.softmax_pmf(np.zeros((3, 256))), 1 / 256, rtol=0, atol=1e-15)
    o = np.zeros((1, 256))
    o[0, 77] = 200.0
    p = sm.softmax_pmf(o)
    assert abs(p[0, 77] - 1.0) < 1e-15 and p.sum() == pytest.approx(1.0, abs=1e-14)
    rng = np.random.default_rng(2)
    p = sm.softmax_pmf(rng.normal(0, 4, (20, 256)))
    assert np.all(p >= 0) and np.allclose(p.sum(axis=1), 1.0, atol=1e-12)


def test_table_rule_equal_logits_closed_form():
    # e = 1, S = 256, r = 2^-8, C_v = v / 256 exactly: F(v) = v + 255 v = 256 v
    F = sm.table_softmax32(np.full((2, 256), 3.25, np.float32))
    assert np.array_equal(F[0], 256 * np.arange(257))
    assert np.array_equal(F[1], F[0])


@pytest.mark.parametrize("k", [0, 63, 64, 130, 255])
def test_table_rule_dominant_level_closed_form(k):
    # exp(-120) ~ 7.7e-53 rounds to 0 in FP32: p_k = 1, C = 0 up to k and 1 after,
    # so f_k = 1 + M' and every other level keeps its floor of 1
    o = np.zeros((1, 256), np.float32)
    o[0, k] = 120.0
    F = sm.table_softmax32(o)[0]
    f = np.diff(F)
    assert f[k] == 1 + oracle.M_PRIME and np.all(np.delete(f, k) == 1)


def test_table_rule_valid_and_near_exact():
    rng = np.random.default_rng(3)
    lg = np.concatenate([rng.normal(0, s, (200, 256)) for s in (0.1, 1, 5, 30)])
    lg[0] = 0.0
    lg[1, :] = -1e4
    lg[1, 5] = 1e4                                   # saturated extremes
    lg[2] = np.linspace(-80, 80, 256)                # long tails
    F32 = sm.table_softmax32(lg.astype(np.float32))
    f = np.diff(F32, axis=1)
    assert np.all(F32[:, 0] == 0) and np.all(F32[:, -1] == 65536) and np.all(f >= 1)
    # the FP32 rule stays within 2 counts of the exact FP64 table of the same logits
    Fx = sm.table_softmax_exact(lg.astype(np.float32).astype(np.float64))
    assert np.abs(F32 - Fx).max() <= 2


def test_ideal_bits_direct_sum_and_coded_cost():
    rng = np.random.default_rng(4)
    lg = rng.normal(0, 3, (300, 256))
    v = rng.integers(0, 256, 300)
    p = sm.softmax_pmf(lg)
    direct = -math.fsum(math.log2(p[i, v[i]]) for i in range(300))
    assert sm.ideal_bits_softmax(lg, v) == pytest.approx(direct, rel=1e-12)
    # cost of the exact-rule table: f_v > P(v) M' gives at most log2(M / M') extra per symbol
    F = sm.table_softmax_exact(lg)
    f = F[np.arange(300), v + 1] - F[np.arange(300), v]
    cost = -np.log2(f / 65536.0).sum()
    assert cost <= direct + 300 * math.log2(65536 / 65280) + 1e-9


@pytest.mark.parametrize("h,w,G,L", [(9, 13, 1, 4), (14, 6, 2, 4), (5, 21, 1, 8)])
def test_codec_round_trip(h, w, G, L):
    layers = _layers(H=32, seed=h + w)
    img = synth.synth_image(h, w, 60 + h)
    buf = sm.encode_image_softmax(img, layers, G, L)
    hdr = oracle.parse_header(buf)
    assert hdr["n_mix"] == 0 and hdr["h1"] == 32 and hdr["fingerprint"] == sm.stored_fingerprint(layers)
    assert np.array_equal(sm.decode_image_softmax(buf, layers), img)
    # payload near the ideal length of the same network
    logits = sm.deep_forward_bf16(oracle.causal_features(img).reshape(-1, 12), layers)
    ideal = sm.ideal_bits_softmax(logits, img.reshape(-1))
    payload = 8 * (len(buf) - oracle.HEADER_SIZE - 4 * G)
    assert payload <= ideal + img.size * (math.log2(65536 / 65280) + 0.03) + 32 * G * L


def test_wrong_network_is_refused():
    layers = _layers(H=32, seed=1)
    img = synth.synth_image(6, 7, 1)
    buf = sm.encode_image_softmax(img, layers, 1, 4)
    other = [(W, b + np.float32(0.01)) for W, b in layers]
    with pytest.raises(ValueError):
        sm.decode_image_softmax(buf, other)
