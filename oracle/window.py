"""Causal neighbourhood window and wavefront steps (oracle; test infrastructure).

Paper passages followed:
  * Section II-A and Fig. 1 (left): the density of a target pixel is
    estimated from a neighbourhood window masked to pixels that are already
    decoded; any window shape may be used.
  * Fig. 1 (right) caption: window positions outside the image are
    substituted with dummy values.
  * Section II-B (Preprocessor): wavefront order similar to HEVC WPP; in
    each coding step every pixel whose window is already coded is coded.

Readings where the paper is silent: the window is the
12 causal neighbours of rows y-2 and y-1 at dx = -2..+2 plus (y, x-2) and
(y, x-1), in that row-major order; pixel values are scaled to [-1, 1] by
s(v) = (2v - 255)/255; the dummy value is 0.0 in the scaled domain; the
wavefront step of pixel (y, x) is t = x + 3y.

Parity: pinned by a hand-derived golden window (tests/golden), causality
and step-legality brute force, and the closed-form step count.
"""
from __future__ import annotations

import numpy as np

# (dy, dx) offsets of the causal window, in feature order.
NEIGHBOURS = ((-2, -2), (-2, -1), (-2, 0), (-2, 1), (-2, 2),
              (-1, -2), (-1, -1), (-1, 0), (-1, 1), (-1, 2),
              (0, -2), (0, -1))
K_IN = len(NEIGHBOURS)
# Wavefront skew: pixel (y, x) is coded in step x + SKEW*y.
SKEW = 3
DUMMY = 0.0


def scale(v, depth: int = 8):
    """Map grey levels to [-1, 1]: s(v) = (2v - m)/m with m = 2^depth - 1 (255 for
    8-bit images, 4095 for 12-bit ones), in FP64."""
    m = float((1 << depth) - 1)
    return (2.0 * np.asarray(v, dtype=np.float64) - m) / m


def pixel_features(img: np.ndarray, y: int, x: int, depth: int = 8) -> np.ndarray:
    """Window of one pixel, read one neighbour at a time (FP64, length 12)."""
    h, w = img.shape
    out = np.empty(K_IN, dtype=np.float64)
    for k, (dy, dx) in enumerate(NEIGHBOURS):
        yy, xx = y + dy, x + dx
        if 0 <= yy < h and 0 <= xx < w:
            out[k] = scale(img[yy, xx], depth)
        else:
            out[k] = DUMMY
    return out


def causal_features(img: np.ndarray, depth: int = 8) -> np.ndarray:
    """Windows of every pixel as one matrix, one row per pixel: (h*w, 12) FP64.

    Row order is raster order (row y, then column x).
    """
    h, w = img.shape
    s = scale(img, depth)
    feats = np.full((h, w, K_IN), DUMMY, dtype=np.float64)
    for k, (dy, dx) in enumerate(NEIGHBOURS):
        y0, y1 = max(0, -dy), min(h, h - dy)
        x0, x1 = max(0, -dx), min(w, w - dx)
        if y0 < y1 and x0 < x1:
            feats[y0:y1, x0:x1, k] = s[y0 + dy:y1 + dy, x0 + dx:x1 + dx]
    return feats.reshape(h * w, K_IN)


def step_of(y, x):
    """Wavefront step of pixel (y, x)."""
    return np.asarray(x) + SKEW * np.asarray(y)


def n_steps(h: int, w: int) -> int:
    """Number of wavefront steps: one more than the step of the last pixel."""
    if h <= 0 or w <= 0:
        return 0
    return int(step_of(h - 1, w - 1)) + 1
