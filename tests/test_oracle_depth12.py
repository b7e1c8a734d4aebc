"""Pins of the oracle's 12-bit form of the softmax network (CPU): the input scale at
its ends and middle, the 4096-level table rule against closed forms (equal logits give
F(v) = 16 v exactly, a dominant level gives f = M - 4096 + 1), against the exact FP64
table and validity on random and extreme logits, the rate floor of the 16-bit table, the
stream's depth marker, and round trips of images and volumes."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import softmax as sm
from oracle import volume as vo

N = 4096


def _layers(H=16, seed=5, k_in=12, bias=0.05):
    layers = synth.xavier_deep(H, seed, k_in=k_in, n_out=N)
    rng = np.random.default_rng(seed + 1)
    return [(W, rng.normal(0, bias, b.shape).astype(np.float32)) for W, b in layers]


def test_scale_closed_forms():
    assert oracle.scale(0, 12) == -1.0 and oracle.scale(4095, 12) == 1.0
    assert oracle.scale(2048, 12) == pytest.approx(1.0 / 4095, abs=0)
    # 8-bit unchanged
    assert oracle.scale(255) == 1.0 and oracle.scale(128) == 1.0 / 255


def test_equal_logits_give_sixteen_v():
    # e = 1, every block sums to 64, S = 4096, p = 2^-12, offsets b 2^-6 and running
    # sums k 2^-12 are exact, C_v = v / 4096, C_v (M - N) = 15 v: F(v) = 16 v
    F = sm.table_softmax32(np.full((2, N), -1.5, np.float32))
    assert np.array_equal(F[0], 16 * np.arange(N + 1))
    assert np.array_equal(F[1], F[0])


@pytest.mark.parametrize("k", [0, 63, 64, 2047, 4032, 4095])
def test_dominant_level(k):
    o = np.zeros((1, N), np.float32)
    o[0, k] = 400.0
    F = sm.table_softmax32(o)[0]
    f = np.diff(F)
    assert f[k] == 65536 - N + 1
    assert np.all(np.delete(f, k) == 1)


def test_rule_near_exact_table_and_valid():
    rng = np.random.default_rng(3)
    for scale in (0.5, 4.0, 30.0):
        o = rng.normal(0, scale, (20, N)).astype(np.float32)
        F = sm.table_softmax32(o)
        E = sm.table_softmax_exact(o.astype(np.float64))
        assert np.abs(F - E).max() <= 2
        f = np.diff(F, axis=1)
        assert np.all(f >= 1) and np.all(F[:, -1] == 65536) and np.all(F[:, 0] == 0)
    o = np.full((3, N), -80.0, np.float32)
    o[0, ::7] = 80.0
    o[1, 4000:] = 1e30
    o[2] = np.linspace(-100, 100, N, dtype=np.float32)
    F = sm.table_softmax32(o)
    assert np.all(np.diff(F, axis=1) >= 1) and np.all(F[:, -1] == 65536)


def test_rate_floor_of_the_16_bit_table():
    # one dominant level keeps 61 441 of 65 536 counts: the cost above 0 bits
    o = np.zeros((1, N), np.float32)
    o[0, 9] = 500.0
    F = sm.table_softmax32(o)[0]
    bits = -math.log2((F[10] - F[9]) / 65536)
    assert bits == pytest.approx(-math.log2(15 / 16 + 1 / 65536), rel=1e-12)
    assert bits < 0.0931


def test_network_has_4096_outputs_and_depth_marker():
    layers = _layers()
    assert sm.net_depth(layers) == 12 and sm.header_dtype(12) == 0x41 and sm.header_dtype(8) == 1
    img = synth.mri_volume(4, 1, 12, bits=12)[0][:6, :9]
    buf = sm.encode_image_softmax(img, layers, 1, 2)
    hdr = oracle.parse_header(buf)
    assert hdr["dtype"] == 0x41 and hdr["n_mix"] == 0 and hdr["k_in"] == 12
    # an 8-bit network of the same shape otherwise refuses the stream
    with pytest.raises(ValueError):
        sm.decode_image_softmax(buf, synth.xavier_deep(16, 5))


def test_image_round_trip_and_length():
    layers = _layers(seed=9)
    img = synth.mri_volume(7, 1, 12, bits=12)[0][:7, :10]
    assert img.dtype == np.uint16 and img.max() < N
    buf = sm.encode_image_softmax(img, layers, 2, 2)
    assert np.array_equal(sm.decode_image_softmax(buf, layers), img)
    o = sm.deep_forward_bf16(oracle.causal_features(img, 12).reshape(-1, 12), layers)
    ideal = sm.ideal_bits_softmax(o, img.reshape(-1))
    body = 16 * (len(buf) - oracle.HEADER_SIZE - 8) // 2
    assert ideal <= body <= ideal + img.size * (-math.log2(15 / 16) + 0.02) + 2 * 2 * 32 + 64


def test_volume_round_trip():
    layers = _layers(seed=13, k_in=21)
    vol = synth.mri_volume(12, 2, 8, bits=12)[:, :6, :7]
    buf = vo.encode_volume(vol, layers, 1, 2, 1)
    hdr = oracle.parse_header(buf)
    assert hdr["dtype"] == 0x41 and hdr["k_in"] == 21
    assert np.array_equal(vo.decode_volume(buf, layers), vol)
