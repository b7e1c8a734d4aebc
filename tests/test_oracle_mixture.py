"""Pins of the oracle's discretised logistic mixture (CPU)."""
import math

import numpy as np

import oracle


def _rand_params(rng, n):
    logits = rng.normal(0, 2, size=(n, 5))
    o = np.concatenate([logits, rng.uniform(-1.2, 1.2, (n, 5)), rng.uniform(-7.5, 1.0, (n, 5))], 1)
    return oracle.mixture_head(o)


def test_masses_sum_to_one():
    rng = np.random.default_rng(0)
    pi, mu, inv_s = _rand_params(rng, 50)
    for i in range(50):
        p = oracle.pmf_table(pi[i], mu[i], inv_s[i])
        assert (p >= 0).all()
        assert abs(math.fsum(p) - 1.0) < 1e-12


def test_log_form_matches_direct_difference():
    rng = np.random.default_rng(1)
    pi, mu, inv_s = _rand_params(rng, 30)
    v = np.arange(256)
    for i in range(30):
        p = oracle.pmf_table(pi[i], mu[i], inv_s[i])
        lp = oracle.log_pmf(v, pi[i][None, :], mu[i][None, :], inv_s[i][None, :])
        good = p > 1e-6
        np.testing.assert_allclose(np.exp(lp[good]), p[good], rtol=1e-8)


def test_single_logistic_bin_centred_closed_form():
    # Mean on the centre of bin v: P(v) = sigma(a) - sigma(-a) = tanh(inv_s/510), a = inv_s/255.
    for v in (1, 17, 128, 254):
        for inv_s in (0.5, 3.0, 40.0, math.exp(7)):
            centre = (2 * v - 255) / 255.0
            pi = np.full(5, 0.2)                 # five identical components act as one
            mu = np.full(5, centre)
            s = np.full(5, inv_s)
            p = oracle.pmf_table(pi, mu, s)[v]
            lp = oracle.log_pmf(np.array([v]), pi[None], mu[None], s[None])[0]
            want = math.tanh(inv_s / 510.0)
            assert abs(p - want) <= 1e-12 * max(1.0, want) + 1e-15
            assert abs(math.exp(lp) - want) <= 1e-12 * want


def test_mirror_symmetry_for_zero_means():
    rng = np.random.default_rng(2)
    pi, _, inv_s = _rand_params(rng, 10)
    mu = np.zeros_like(pi)
    v = np.arange(256)
    for i in range(10):
        lp = oracle.log_pmf(v, pi[i][None], mu[i][None], inv_s[i][None])
        np.testing.assert_allclose(lp, lp[::-1], rtol=1e-12, atol=1e-12)


def test_open_end_bins():
    # All mass far below the first edge lands in level 0, far above in level 255.
    pi = np.full(5, 0.2); s = np.full(5, math.exp(7))
    assert oracle.pmf_table(pi, np.full(5, -3.0), s)[0] == 1.0
    assert oracle.pmf_table(pi, np.full(5, 3.0), s)[255] == 1.0


def test_ideal_bits_brute_force(c0_inputs):
    img, w = c0_inputs
    img = img[:9, :11]
    feats = oracle.causal_features(img)
    o = oracle.mlp_forward(feats, w["W1"], w["b1"], w["W2"], w["b2"], w["W3"], w["b3"])
    pi, mu, inv_s = oracle.mixture_head(o)
    brute = math.fsum(-math.log2(oracle.pmf_table(pi[i], mu[i], inv_s[i])[int(v)])
                      for i, v in enumerate(img.ravel()))
    assert abs(oracle.ideal_bits_image(img, w) - brute) < 1e-9 * brute
