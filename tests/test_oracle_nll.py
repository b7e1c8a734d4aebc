"""Pins of the oracle's retraining pieces (CPU): sampled windows, the loss in bits, its
finite-difference gradient and the Adam update.

Each pin compares the oracle with something it does not compute itself: the whole-image
window matrix (pinned by the hand-derived goldens), a per-sample loop over CDF differences,
closed-form derivatives of a single logistic, the softmax shift invariance, and
torch.optim.Adam.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth

LN2 = math.log(2.0)


def _tiny_stack(n=3, h=7, w=9, seed=0):
    return np.random.default_rng(seed).integers(0, 256, size=(n, h, w)).astype(np.uint8)


def _all_indices(n, h, w):
    s, y, x = np.meshgrid(np.arange(n), np.arange(h), np.arange(w), indexing="ij")
    return np.stack([s.ravel(), y.ravel(), x.ravel()], axis=1).astype(np.int32)


def test_sample_features_are_the_slice_windows():
    stack = _tiny_stack()
    n, h, w = stack.shape
    idx = _all_indices(n, h, w)
    got = oracle.sample_features(stack, idx)
    for s in range(n):
        ref = oracle.causal_features(stack[s])  # pinned by tests/golden/window_3x3.txt
        for y in range(h):
            for x in range(w):
                row = got[(s * h + y) * w + x]
                assert np.array_equal(row, ref[y * w + x]), (s, y, x)
    # windows never cross from one slice into the next
    one = np.array([[1, 0, 0]], np.int32)
    assert np.all(oracle.sample_features(stack, one) == 0.0)


def test_sample_features_repeated_and_unordered_indices():
    stack = _tiny_stack(seed=1)
    idx = np.array([[2, 6, 8], [0, 0, 0], [2, 6, 8], [1, 3, 1]], np.int32)
    got = oracle.sample_features(stack, idx)
    for r, (s, y, x) in enumerate(idx):
        assert np.array_equal(got[r], oracle.pixel_features(stack[s], int(y), int(x)))


def _brute_loss(weights, stack, idx):
    """Mean of -log2 P(target) by a loop over samples, P from CDF differences."""
    tot = []
    for s, y, x in idx:
        f = oracle.pixel_features(stack[s], int(y), int(x))[None, :]
        o = oracle.mlp_forward(f, *(weights[k] for k in oracle.PARAM_ORDER))
        pi, mu, inv_s = oracle.mixture_head(o)
        p = oracle.pmf_table(pi[0], mu[0], inv_s[0])
        tot.append(-math.log2(p[int(stack[s, y, x])]))
    return math.fsum(tot) / len(tot)


def test_nll_bits_equals_brute_force_mean():
    stack = synth.mri_stack(2000, 2)
    idx = synth.train_indices(5, 300, len(stack), 256, 256)
    w = synth.xavier_mlp((12, 32, 32, 15), 3)
    got = oracle.nll_bits(w, stack, idx)
    ref = _brute_loss(w, stack, idx)
    assert abs(got - ref) < 1e-10 * ref
    # the mean is over samples: duplicating every sample leaves it unchanged
    assert abs(oracle.nll_bits(w, stack, np.concatenate([idx, idx])) - got) < 1e-12 * got


def _constant_output_weights(mu, log_s, hidden=8, b2=None):
    """W = 0 everywhere, so every pixel gets o = b3: five identical components."""
    w = {"W1": np.zeros((hidden, 12)), "b1": np.zeros(hidden),
         "W2": np.zeros((hidden, hidden)), "b2": np.zeros(hidden) if b2 is None else b2,
         "W3": np.zeros((15, hidden)), "b3": np.zeros(15)}
    w["b3"][5:10] = mu
    w["b3"][10:15] = log_s
    return w


def _sig(t):
    return 1.0 / (1.0 + math.exp(-t)) if t >= 0 else math.exp(t) / (1.0 + math.exp(t))


def _single_logistic_derivs(v, mu, log_s):
    """P(v) of one logistic and dP/dmu, dP/dlog_s written out by hand."""
    s = math.exp(-log_s)
    hi = (2 * v + 1) / 255.0 - 1.0
    lo = (2 * v - 1) / 255.0 - 1.0

    def parts(beta, end):
        if end:  # an open end: sigma is constant there, its derivatives vanish
            return 0.0, 0.0
        t = (beta - mu) * s
        d = _sig(t) * (1.0 - _sig(t))
        return d, t * d
    dA, tA = parts(hi, v == 255)
    dB, tB = parts(lo, v == 0)
    SA = 1.0 if v == 255 else _sig((hi - mu) * s)
    SB = 0.0 if v == 0 else _sig((lo - mu) * s)
    P = SA - SB
    dP_dmu = -s * (dA - dB)
    dP_dls = -(tA - tB)
    return P, dP_dmu, dP_dls


def test_fd_gradient_matches_single_logistic_closed_form():
    stack = _tiny_stack(n=2, h=6, w=5, seed=3)
    idx = _all_indices(2, 6, 5)
    mu, log_s = 0.1, -2.5
    w = _constant_output_weights(mu, log_s)
    tg = stack[idx[:, 0], idx[:, 1], idx[:, 2]].astype(int)
    P = np.array([_single_logistic_derivs(int(v), mu, log_s) for v in tg])
    loss_ref = float(np.mean(-np.log2(P[:, 0])))
    # one mixture component k carries weight 1/5 of every derivative
    g_mu = float(np.mean(-(P[:, 1] / P[:, 0]) / LN2)) / 5.0
    g_ls = float(np.mean(-(P[:, 2] / P[:, 0]) / LN2)) / 5.0
    picks = [("b3", k) for k in range(15)]
    loss, fd = oracle.nll_and_grad_fd(w, stack, idx, picks, h=1e-6)
    assert abs(loss - loss_ref) < 1e-12 * loss_ref
    assert np.allclose(fd[0:5], 0.0, atol=1e-8)          # identical components: no logit pull
    assert np.allclose(fd[5:10], g_mu, rtol=1e-6, atol=0)
    assert np.allclose(fd[10:15], g_ls, rtol=1e-6, atol=0)


def test_fd_gradient_chain_through_last_layer():
    # W1 = W2 = 0 and b2 > 0 give a constant hidden vector h2 = b2, so
    # d loss / d W3[j, i] = d loss / d b3[j] * b2[i]: a transposed or shifted index fails.
    stack = _tiny_stack(n=1, h=5, w=6, seed=4)
    idx = _all_indices(1, 5, 6)
    b2 = np.array([0.5, 1.25, 2.0, 0.75])
    w = _constant_output_weights(-0.2, -3.0, hidden=4, b2=b2)
    picks_b = [("b3", j) for j in (5, 11)]
    picks_w = [("W3", 4 * j + i) for j in (5, 11) for i in range(4)]
    _, gb = oracle.nll_and_grad_fd(w, stack, idx, picks_b, h=1e-6)
    _, gw = oracle.nll_and_grad_fd(w, stack, idx, picks_w, h=1e-6)
    ref = np.array([gb[a] * b2[i] for a in range(2) for i in range(4)])
    assert np.allclose(gw, ref, rtol=1e-6, atol=1e-10)


def test_fd_gradient_softmax_gauge():
    # adding one constant to all five logits leaves the loss unchanged
    stack = synth.mri_stack(2010, 1)
    idx = synth.train_indices(7, 200, 1, 256, 256)
    w = synth.xavier_mlp((12, 32, 32, 15), 9)
    w = {k: np.asarray(v, np.float64) for k, v in w.items()}
    w["b3"] = np.random.default_rng(2).normal(0, 0.3, 15)
    _, fd = oracle.nll_and_grad_fd(w, stack, idx, [("b3", k) for k in range(5)], h=1e-6)
    assert abs(fd.sum()) < 1e-8 * np.abs(fd).sum() + 1e-9
    assert np.abs(fd).max() > 1e-3  # the gauge is not trivially zero


@pytest.mark.parametrize("shape", [(7,), (4, 3)])
def test_adam_update_matches_torch_optim(shape):
    rng = np.random.default_rng(11)
    p0 = rng.normal(0, 1, shape)
    ref = torch.from_numpy(p0.copy()).requires_grad_(True)
    opt = torch.optim.Adam([ref], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    p, m, v = p0.copy(), np.zeros(shape), np.zeros(shape)
    for step in range(1, 6):
        g = rng.normal(0, 10.0 ** rng.integers(-4, 2), shape)
        ref.grad = torch.from_numpy(g.copy())
        opt.step()
        p, m, v = oracle.adam_update(p, g, m, v, step)
        assert np.allclose(p, ref.detach().numpy(), rtol=1e-13, atol=1e-15), step
    # first step from zero moments moves every parameter by lr against the gradient's sign
    p1, _, _ = oracle.adam_update(p0, np.full(shape, 3.0), np.zeros(shape), np.zeros(shape), 1)
    assert np.allclose(p0 - p1, 1e-3, rtol=1e-6)
