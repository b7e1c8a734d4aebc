"""Pins of the oracle's network and mixture head (CPU)."""
import numpy as np
import torch

import oracle
import synth


def test_zero_weights_give_output_bias():
    w = synth.xavier_mlp((12, 8, 8, 15), 1)
    for k in ("W1", "W2", "W3"):
        w[k] = np.zeros_like(w[k])
    w["b3"] = np.arange(15, dtype=np.float32) - 7
    f = np.random.default_rng(0).uniform(-1, 1, size=(10, 12))
    o = oracle.mlp_forward(f, w["W1"], w["b1"], w["W2"], w["b2"], w["W3"], w["b3"])
    assert np.array_equal(o, np.broadcast_to(w["b3"].astype(np.float64), (10, 15)))


def test_one_hidden_unit_hand_example():
    W1 = np.zeros((1, 12)); W1[0, 0] = 0.5; W1[0, 11] = -1.0
    b1 = np.array([0.25]); W2 = np.array([[2.0]]); b2 = np.array([-0.5])
    W3 = (np.arange(1, 16) / 10.0)[:, None]; b3 = np.zeros(15)
    f = np.zeros((2, 12)); f[0, 0] = 0.2; f[0, 11] = -0.6; f[1, 0] = 0.2; f[1, 11] = 1.0
    o = oracle.mlp_forward(f, W1, b1, W2, b2, W3, b3)
    # h1 = relu(0.1 + 0.6 + 0.25) = 0.95, h2 = relu(1.9 - 0.5) = 1.4 ; second row is cut by ReLU
    np.testing.assert_allclose(o[0], 1.4 * np.arange(1, 16) / 10.0, rtol=1e-15, atol=1e-15)
    assert (o[1] == 0.0).all()


def test_mlp_matches_torch_fp64_chain():
    w = synth.xavier_mlp((12, 64, 64, 15), 3)
    w["b1"] = np.linspace(-0.2, 0.2, 64).astype(np.float32)
    w["b2"] = np.linspace(0.1, -0.1, 64).astype(np.float32)
    w["b3"] = np.linspace(-1, 1, 15).astype(np.float32)
    f = np.random.default_rng(1).uniform(-1, 1, size=(257, 12))
    o = oracle.mlp_forward(f, w["W1"], w["b1"], w["W2"], w["b2"], w["W3"], w["b3"])
    T = {k: torch.from_numpy(v.astype(np.float64)) for k, v in w.items()}
    x = torch.from_numpy(f)
    ref = torch.nn.functional.linear(x, T["W1"], T["b1"]).relu()
    ref = torch.nn.functional.linear(ref, T["W2"], T["b2"]).relu()
    ref = torch.nn.functional.linear(ref, T["W3"], T["b3"])
    np.testing.assert_allclose(o, ref.numpy(), rtol=1e-12, atol=1e-12)


def test_head_softmax_and_clamp():
    o = np.zeros((3, 15))
    o[0, 0:5] = [1000.0, 0.0, -5.0, 2.0, 3.0]
    o[1, 10:15] = [-10.0, -7.0, 0.0, 1.0, 7.0]
    o[2, 0:5] = np.log([0.1, 0.2, 0.3, 0.15, 0.25])
    pi, mu, inv_s = oracle.mixture_head(o)
    np.testing.assert_allclose(pi.sum(axis=1), 1.0, rtol=0, atol=1e-15)
    assert pi[0, 0] == 1.0
    np.testing.assert_allclose(pi[2], [0.1, 0.2, 0.3, 0.15, 0.25], rtol=1e-14)
    np.testing.assert_allclose(inv_s[1], np.exp([7.0, 7.0, 0.0, -1.0, -7.0]), rtol=1e-15)
    assert (mu == 0).all()
