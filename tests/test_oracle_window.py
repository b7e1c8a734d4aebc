"""Pins of the oracle's causal window and wavefront steps (CPU)."""
import itertools

import numpy as np

import oracle
from oracle.window import NEIGHBOURS


def test_golden_window(golden):
    lines = golden("window_3x3.txt")
    img = np.array([[int(v) for v in ln.split()[1:]] for ln in lines if ln.startswith("image")],
                   dtype=np.uint8)
    feats = oracle.causal_features(img).reshape(3, 3, 12)
    n = 0
    for ln in lines:
        if not ln.startswith("pixel"):
            continue
        head, vals = ln.split(":")
        _, y, x = head.split()
        want = np.array([float(v) for v in vals.split()])
        np.testing.assert_allclose(feats[int(y), int(x)], want, rtol=0, atol=1e-15)
        np.testing.assert_allclose(oracle.pixel_features(img, int(y), int(x)), want,
                                   rtol=0, atol=1e-15)
        n += 1
    assert n == 4


def test_scale_endpoints_and_dummy():
    assert oracle.scale(0) == -1.0 and oracle.scale(255) == 1.0
    img = np.full((1, 1), 200, np.uint8)
    assert (oracle.causal_features(img) == 0.0).all()


def test_window_is_causal_brute_force():
    # Changing any pixel at or after (y, x) in step order never changes the window of (y, x).
    rng = np.random.default_rng(0)
    for h, w in ((5, 7), (4, 3), (1, 6), (6, 1)):
        img = rng.integers(0, 256, size=(h, w)).astype(np.uint8)
        base = oracle.causal_features(img).reshape(h, w, 12)
        for y, x in itertools.product(range(h), range(w)):
            t = oracle.step_of(y, x)
            for yy, xx in itertools.product(range(h), range(w)):
                if oracle.step_of(yy, xx) < t:
                    continue
                mod = img.copy()
                mod[yy, xx] = 255 - mod[yy, xx]
                got = oracle.pixel_features(mod, y, x)
                assert np.array_equal(got, base[y, x]), (h, w, y, x, yy, xx)


def test_every_neighbour_is_in_an_earlier_step():
    dts = [dx + oracle.SKEW * dy for dy, dx in NEIGHBOURS]
    assert max(dts) <= -1 and min(dts) >= -8
    # With a skew of 2 the up-right neighbour would share the pixel's step.
    assert any(dx + 2 * dy == 0 for dy, dx in NEIGHBOURS)


def test_step_count_closed_form():
    for h, w in ((1, 1), (64, 64), (1536, 2048), (7, 3), (3, 7)):
        assert oracle.n_steps(h, w) == w + 3 * h - 3
    for h, w in ((5, 7), (9, 2), (2, 9)):
        yy, xx = np.mgrid[0:h, 0:w]
        t = oracle.step_of(yy, xx).ravel()
        counts = np.bincount(t, minlength=oracle.n_steps(h, w))
        assert counts.sum() == h * w and len(counts) == oracle.n_steps(h, w)
        if w >= oracle.SKEW:
            assert (counts >= 1).all()
        assert counts.max() <= min(h, -(-w // oracle.SKEW))
