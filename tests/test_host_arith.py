"""Arithmetic identities that the decoder kernels rely on, checked exactly on the CPU.

The decoder computes the bin edge beta_v = RN((2v - 256) / 255) (the FP32 edges of the
256 grey levels, Section II-B's discretisation) and the scaled grey level RN((2v - 255) / 255)
of a window feature as one product by RN(1/255) and two fused corrections instead of reading
the tables.  This must equal the correctly rounded quotient for every level, or encoder and
decoder would disagree on a frequency.
"""
from fractions import Fraction

import numpy as np


def _rn32(fr: Fraction) -> np.float32:
    """Round an exact rational to the nearest float32, ties to even."""
    f = np.float32(float(fr))
    cands = [np.nextafter(f, np.float32(-np.inf)), f, np.nextafter(f, np.float32(np.inf))]

    def key(c):
        return (abs(Fraction(float(c)) - fr), int(np.float32(c).view(np.uint32)) & 1)

    return np.float32(min(cands, key=key))


def _fma32(a, b, c) -> np.float32:
    return _rn32(Fraction(float(a)) * Fraction(float(b)) + Fraction(float(c)))


def test_bin_edge_by_reciprocal_and_two_fmas_is_the_rounded_quotient():
    r = np.float32(1.0) / np.float32(255.0)
    for v in range(1, 256):
        xv = np.float32(2 * v - 256)
        want = _rn32(Fraction(2 * v - 256, 255))
        assert want == np.float32(xv / np.float32(255.0))      # numpy's division agrees
        q0 = np.float32(xv * r)
        e = _fma32(-q0, np.float32(255.0), xv)
        got = _fma32(e, r, q0)
        assert got == want, v


def test_reciprocal_and_two_fmas_give_every_quotient_by_255_in_range():
    # every integer numerator in [-256, 256]: the bin edges (2v - 256) and the
    # scaled grey levels (2v - 255) of the window features
    r = np.float32(1.0) / np.float32(255.0)
    for n in range(-256, 257):
        xv = np.float32(n)
        q0 = np.float32(xv * r)
        e = _fma32(-q0, np.float32(255.0), xv)
        assert _fma32(e, r, q0) == _rn32(Fraction(n, 255)), n


def test_plain_reciprocal_product_alone_is_not_enough():
    # the corrections are needed: the bare product misses for many levels
    r = np.float32(1.0) / np.float32(255.0)
    misses = sum(np.float32(np.float32(2 * v - 256) * r) != _rn32(Fraction(2 * v - 256, 255))
                 for v in range(1, 256))
    assert misses > 0
