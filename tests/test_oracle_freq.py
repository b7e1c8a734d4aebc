"""Pins of the oracle's frequency quantisation (CPU)."""
import math

import numpy as np

import oracle

M, MP = oracle.M_TOTAL, oracle.M_PRIME


def _params(rng, n, extreme=False):
    lo = -7.5 if extreme else -4.0
    o = np.concatenate([rng.normal(0, 3 if extreme else 1, (n, 5)),
                        rng.uniform(-1.5, 1.5, (n, 5)), rng.uniform(lo, 2.0, (n, 5))], 1)
    return oracle.mixture_head(o)


def test_exact_tables_valid_and_bounded():
    rng = np.random.default_rng(0)
    pi, mu, inv_s = _params(rng, 200, extreme=True)
    for i in range(200):
        F = oracle.table_exact(pi[i], mu[i], inv_s[i])
        f = np.diff(F)
        assert F[0] == 0 and F[-1] == M and f.sum() == M and f.min() >= 1
        P = oracle.pmf_table(pi[i], mu[i], inv_s[i])
        # f_v = 1 + q_{v+1} - q_v with q = floor(C M'): P M' < f < P M' + 2.
        assert (f > P * MP - 1e-9).all() and (f < P * MP + 2 + 1e-9).all()


def test_fp32_tables_valid_for_wild_parameters():
    rng = np.random.default_rng(1)
    for extreme in (False, True):
        pi, mu, inv_s = _params(rng, 300, extreme)
        F = oracle.table_full32(pi.astype(np.float32), mu.astype(np.float32), inv_s.astype(np.float32))
        f = np.diff(F, axis=1)
        assert (F[:, 0] == 0).all() and (F[:, -1] == M).all()
        assert (f >= 1).all() and (f.sum(axis=1) == M).all()


def test_fp32_table_close_to_exact_table():
    rng = np.random.default_rng(2)
    pi, mu, inv_s = _params(rng, 100)
    F32 = oracle.table_full32(pi.astype(np.float32), mu.astype(np.float32), inv_s.astype(np.float32))
    for i in range(100):
        F64 = oracle.table_exact(pi[i], mu[i], inv_s[i])
        assert np.abs(F32[i] - F64).max() <= 2


def test_levels_rule_equals_full_table():
    rng = np.random.default_rng(3)
    pi, mu, inv_s = (a.astype(np.float32) for a in _params(rng, 64))
    full = oracle.table_full32(pi, mu, inv_s)
    lv = rng.integers(0, 257, size=(64, 7))
    got = oracle.table_levels32(lv, pi, mu, inv_s)
    assert np.array_equal(got, np.take_along_axis(full, lv, axis=1))


def test_sigma_lut_knots_and_slopes():
    S, D = oracle.sigma_lut32()
    assert S.dtype == np.float32 and len(S) == 4097
    t = -16.0 + np.arange(4097) / 128.0
    exact = np.array([1.0 / (1.0 + math.exp(-x)) for x in t])
    # knots are the FP32 roundings of the logistic: within half an ulp
    ulp = np.spacing(S.astype(np.float32)).astype(np.float64)
    assert (np.abs(S.astype(np.float64) - exact) <= 0.5 * ulp + 1e-300).all()
    assert (np.diff(S) >= 0).all()
    # slopes are exact differences, so a segment ends exactly on the next knot
    assert np.array_equal((S[:-1] + D[:-1]).astype(np.float32), S[1:])
    assert D[-1] == 0


def test_sigma_hat_monotone_and_accurate():
    knots = np.arange(4097).astype(np.float32)
    near = np.concatenate([np.nextafter(knots, np.float32(-np.inf)), knots,
                           np.nextafter(knots, np.float32(np.inf))])
    u = np.sort(np.concatenate([near, np.linspace(-3000, 7000, 400001).astype(np.float32),
                                np.array([-np.inf, np.inf], np.float32)]))
    s = oracle.sigma_hat32(u)
    assert (np.diff(s) >= 0).all()
    fin = np.isfinite(u) & (u >= 0) & (u <= 4096)
    t = u[fin].astype(np.float64) / 128.0 - 16.0
    exact = 1.0 / (1.0 + np.exp(-t))
    assert np.abs(s[fin] - exact).max() < 1e-6


def test_table_coordinate_tracks_the_logistic_argument():
    # u = beta A + B is (beta - mu) inv_s on the table's scale, up to FP32 rounding
    rng = np.random.default_rng(4)
    mu = rng.uniform(-1.5, 1.5, 1000).astype(np.float32)
    inv_s = np.exp(rng.uniform(-2, 7, 1000)).astype(np.float32)
    A, B = oracle.table_coords32(mu, inv_s)
    beta = oracle.beta32()[rng.integers(1, 256, 1000)]
    u = beta * A + B
    exact = (beta.astype(np.float64) - mu) * inv_s * 128.0 + 2048.0
    assert np.all(np.abs(u - exact) <= 4 * np.spacing(np.maximum(np.abs(beta * A), np.abs(B))) + 1e-3)


def test_fp32_constants_are_roundings_of_exact_values():
    b = oracle.beta32()
    v = np.arange(1, 256)
    assert np.array_equal(b[1:256], ((2.0 * v - 256) / 255.0).astype(np.float32))
    assert b[0] == -np.inf and b[256] == np.inf
    s = oracle.scale32()
    assert np.array_equal(s, oracle.scale(np.arange(256)).astype(np.float32))
