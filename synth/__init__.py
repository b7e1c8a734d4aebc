"""Seeded synthetic inputs for the DLIC hot path.

This module draws inputs only: greyscale photo-like images, MRI-like phantom
slices, Glorot-initialised network weights, valid frequency tables for coder
tests, and training sample indices.  It contains none of the codec's own
arithmetic (no scaling, no network evaluation, no mixture, no quantisation,
no rANS), so the CPU oracle and the GPU path can both take their inputs from
it without sharing any computation.

The paper measures on the CLIC 2019 mobile set (Section III-A) and on
proprietary 12-bit MRI scans (Section IV-A); neither is available, so these
generators stand in for them.  No item of either dataset is reproduced.
"""
from __future__ import annotations

import numpy as np
from scipy.ndimage import gaussian_filter1d

__all__ = [
    "synth_image",
    "mri_phantom",
    "mri_stack",
    "xavier_mlp",
    "batch_sizes",
    "train_indices",
    "random_tables",
    "random_symbols_from_tables",
    "C3_SIZES",
]

# (h, w) choices for the 64-image batch workload, drawn per image seed.
C3_SIZES = ((256, 256), (384, 512), (768, 1024), (1536, 2048))


def synth_image(h: int, w: int, seed: int) -> np.ndarray:
    """Photo-like 8-bit greyscale image, shape (h, w), dtype uint8.

    Recipe (fixed by seed): a mid-grey field plus three Gaussian-blurred
    white-noise octaves (sigma 2, 8, 24 px; amplitudes 12, 20, 32 grey
    levels after normalising each octave to zero sample mean and unit
    sample std), four random
    straight step edges of height U(-48, 48), and N(0, 3^2) pixel noise;
    rounded half-to-even and clipped to 0..255.
    """
    if h <= 0 or w <= 0:
        raise ValueError("image dimensions must be positive")
    rng = np.random.default_rng(seed)
    field = np.full((h, w), 128.0, dtype=np.float64)
    for sigma, amp in ((2.0, 12.0), (8.0, 20.0), (24.0, 32.0)):
        noise = rng.standard_normal((h, w))
        if h > 1:
            noise = gaussian_filter1d(noise, sigma, axis=0, mode="reflect", truncate=4.0)
        if w > 1:
            noise = gaussian_filter1d(noise, sigma, axis=1, mode="reflect", truncate=4.0)
        noise = noise - noise.mean()
        sd = noise.std()
        if sd > 0:
            field += amp * noise / sd
    yy, xx = np.mgrid[0:h, 0:w].astype(np.float64)
    for _ in range(4):
        px = rng.uniform(0.0, w)
        py = rng.uniform(0.0, h)
        theta = rng.uniform(0.0, np.pi)
        step = rng.uniform(-48.0, 48.0)
        side = (xx - px) * np.cos(theta) + (yy - py) * np.sin(theta) >= 0.0
        field += np.where(side, step, 0.0)
    field += rng.normal(0.0, 3.0, size=(h, w))
    return np.clip(np.rint(field), 0, 255).astype(np.uint8)


def _paint_ellipse(img, cy, cx, a, b, ang, value):
    n = img.shape[0]
    yy, xx = np.mgrid[0:n, 0:n].astype(np.float64)
    dy, dx = yy - cy, xx - cx
    c, s = np.cos(ang), np.sin(ang)
    u = dx * c + dy * s
    v = -dx * s + dy * c
    inside = (u / a) ** 2 + (v / b) ** 2 <= 1.0
    img[inside] = value


def mri_phantom(seed: int, size: int = 256) -> np.ndarray:
    """MRI-like 8-bit slice, shape (size, size), dtype uint8.

    Recipe: 3-8 nested ellipses of random intensity 20-220 on a zero
    background, a smooth multiplicative quadratic bias field, Rician noise
    with sigma 4, rounded and clipped to 0..255.
    """
    rng = np.random.default_rng(seed)
    n_ell = int(rng.integers(3, 9))
    img = np.zeros((size, size), dtype=np.float64)
    half = size / 2.0
    cy = half + rng.uniform(-10.0, 10.0)
    cx = half + rng.uniform(-10.0, 10.0)
    scale = size / 256.0
    a = rng.uniform(70.0, 115.0) * scale
    b = rng.uniform(70.0, 115.0) * scale
    ang = rng.uniform(0.0, np.pi)
    _paint_ellipse(img, cy, cx, a, b, ang, rng.uniform(20.0, 220.0))
    for _ in range(n_ell - 1):
        na = a * rng.uniform(0.45, 0.85)
        nb = b * rng.uniform(0.45, 0.85)
        ou = rng.uniform(-1.0, 1.0) * 0.5 * (a - na)
        ov = rng.uniform(-1.0, 1.0) * 0.5 * (b - nb)
        c, s = np.cos(ang), np.sin(ang)
        cx, cy = cx + ou * c - ov * s, cy + ou * s + ov * c
        ang = ang + rng.uniform(-0.5, 0.5)
        a, b = na, nb
        _paint_ellipse(img, cy, cx, a, b, ang, rng.uniform(20.0, 220.0))
    coef = rng.normal(0.0, 0.5, size=5)
    vv, uu = np.mgrid[0:size, 0:size].astype(np.float64)
    uu = uu / (size - 1) * 2.0 - 1.0
    vv = vv / (size - 1) * 2.0 - 1.0
    bias = np.exp(0.3 * (coef[0] * uu + coef[1] * vv + coef[2] * uu * uu
                         + coef[3] * vv * vv + coef[4] * uu * vv))
    n1 = rng.normal(0.0, 4.0, size=(size, size))
    n2 = rng.normal(0.0, 4.0, size=(size, size))
    mag = np.sqrt((img * bias + n1) ** 2 + n2 ** 2)
    return np.clip(np.rint(mag), 0, 255).astype(np.uint8)


def mri_stack(first_seed: int = 2000, n: int = 256, size: int = 256) -> np.ndarray:
    """Stack of n phantom slices, seeds first_seed..first_seed+n-1, (n, size, size) uint8."""
    return np.stack([mri_phantom(first_seed + k, size) for k in range(n)])


def xavier_mlp(dims, seed: int) -> dict:
    """Glorot-uniform weights for a fully connected net, FP32, biases zero.

    dims = (k_in, h1, h2, n_out).  Draw order W1, W2, W3, each of shape
    [out, in], uniform on +-sqrt(6 / (fan_in + fan_out)), drawn in FP64 from
    numpy's PCG64 and rounded to FP32.
    """
    k_in, h1, h2, n_out = (int(d) for d in dims)
    rng = np.random.default_rng(seed)
    out = {}
    for name, (fo, fi) in (("W1", (h1, k_in)), ("W2", (h2, h1)), ("W3", (n_out, h2))):
        lim = np.sqrt(6.0 / (fi + fo))
        out[name] = rng.uniform(-lim, lim, size=(fo, fi)).astype(np.float32)
    out["b1"] = np.zeros(h1, np.float32)
    out["b2"] = np.zeros(h2, np.float32)
    out["b3"] = np.zeros(n_out, np.float32)
    return out


def xavier_deep(hidden: int, seed: int, depth: int = 6, k_in: int = 12, n_out: int = 256) -> list:
    """Glorot-uniform weights of a dense net k_in -> hidden x (depth - 1) -> n_out, FP32,
    biases zero: [(W, b)] per layer, W of shape [out, in], drawn in layer order from
    numpy's PCG64 as for xavier_mlp."""
    dims = [k_in] + [hidden] * (depth - 1) + [n_out]
    rng = np.random.default_rng(seed)
    out = []
    for fi, fo in zip(dims[:-1], dims[1:]):
        lim = np.sqrt(6.0 / (fi + fo))
        out.append((rng.uniform(-lim, lim, size=(fo, fi)).astype(np.float32),
                    np.zeros(fo, np.float32)))
    return out


def batch_sizes(seeds) -> list:
    """(h, w) per image of the batch workload: one uniform draw from C3_SIZES per seed."""
    return [C3_SIZES[int(np.random.default_rng(s).integers(0, 4))] for s in seeds]


def train_indices(step: int, n: int, n_slices: int, h: int, w: int) -> np.ndarray:
    """Uniform (slice, y, x) samples with replacement for one training step, (n, 3) int32."""
    rng = np.random.default_rng(10_000 + step)
    sl = rng.integers(0, n_slices, size=n)
    yy = rng.integers(0, h, size=n)
    xx = rng.integers(0, w, size=n)
    return np.stack([sl, yy, xx], axis=1).astype(np.int32)


def random_tables(n_tables: int, seed: int, kind: str = "mixed",
                  total: int = 1 << 16, n_sym: int = 256) -> np.ndarray:
    """Valid cumulative frequency tables for coder tests, (n_tables, n_sym+1) uint32.

    Every table starts at 0, ends at `total`, and every symbol has frequency
    >= 1.  kind: 'uniform' (all equal), 'peaked' (one symbol takes all the
    spare mass), 'dirichlet' (random), or 'mixed' (a blend of the three plus
    single-spike tables).
    """
    rng = np.random.default_rng(seed)
    spare = total - n_sym
    tabs = np.empty((n_tables, n_sym + 1), dtype=np.int64)
    for i in range(n_tables):
        k = kind
        if kind == "mixed":
            k = ("uniform", "peaked", "dirichlet", "dirichlet", "sparse")[i % 5]
        if k == "uniform":
            freq = np.full(n_sym, total // n_sym, dtype=np.int64)
            freq[: total - freq.sum()] += 1
        elif k == "peaked":
            freq = np.ones(n_sym, dtype=np.int64)
            freq[int(rng.integers(0, n_sym))] += spare
        elif k == "sparse":
            freq = np.ones(n_sym, dtype=np.int64)
            picks = rng.integers(0, n_sym, size=4)
            share = rng.multinomial(spare, [0.25] * 4)
            for p, s in zip(picks, share):
                freq[p] += s
        else:
            p = rng.dirichlet(np.full(n_sym, 0.3))
            freq = 1 + rng.multinomial(spare, p)
        tabs[i, 0] = 0
        tabs[i, 1:] = np.cumsum(freq)
    assert (tabs[:, -1] == total).all()
    return tabs.astype(np.uint32)


def random_symbols_from_tables(tables: np.ndarray, idx: np.ndarray, seed: int) -> np.ndarray:
    """Draw one symbol per position from its table's distribution (uint8, idx's shape)."""
    rng = np.random.default_rng(seed)
    flat = idx.ravel()
    u = rng.integers(0, int(tables[0, -1]), size=flat.size)
    sym = np.empty(flat.size, dtype=np.uint8)
    for t in np.unique(flat):
        sel = flat == t
        sym[sel] = np.searchsorted(tables[t], u[sel], side="right") - 1
    return sym.reshape(idx.shape)


def mri_volume(seed: int, depth: int = 35, size: int = 256, bits: int = 8) -> np.ndarray:
    """MRI-like volume whose slices are cuts through one 3-D object, shape
    (depth, size, size): uint8 for 8-bit samples (a 256x256x35 scan by default),
    uint16 for 12-bit ones (intensities and noise scaled by 4095/255).

    Recipe: 3-8 nested ellipsoids of random intensity 20-220 on a zero
    background (semi-axes 70-115 px in-plane, 0.6-1.2 times the depth along
    the slice axis, each inner one 0.45-0.85 of its parent, offset inside it),
    a smooth multiplicative quadratic bias field over the volume, Rician noise
    with sigma 4, rounded and clipped to 0..255.  Neighbouring slices are
    strongly but not perfectly alike, as in a scan with a slice gap.
    """
    rng = np.random.default_rng(seed)
    scale = size / 256.0
    zz, yy, xx = np.meshgrid(np.arange(depth, dtype=np.float64) + 0.5,
                             np.arange(size, dtype=np.float64),
                             np.arange(size, dtype=np.float64), indexing="ij")
    vol = np.zeros((depth, size, size), dtype=np.float64)
    c = np.array([depth / 2.0 + rng.uniform(-0.1, 0.1) * depth,
                  size / 2.0 + rng.uniform(-10.0, 10.0), size / 2.0 + rng.uniform(-10.0, 10.0)])
    ax = np.array([rng.uniform(0.6, 1.2) * depth, rng.uniform(70.0, 115.0) * scale,
                   rng.uniform(70.0, 115.0) * scale])
    ang = rng.uniform(0.0, np.pi)
    for i in range(int(rng.integers(3, 9))):
        if i > 0:
            na = ax * rng.uniform(0.45, 0.85, size=3)
            c = c + rng.uniform(-1.0, 1.0, size=3) * 0.5 * (ax - na)
            ax = na
            ang = ang + rng.uniform(-0.5, 0.5)
        dy, dx = yy - c[1], xx - c[2]
        u = dx * np.cos(ang) + dy * np.sin(ang)
        v = -dx * np.sin(ang) + dy * np.cos(ang)
        inside = ((zz - c[0]) / ax[0]) ** 2 + (u / ax[2]) ** 2 + (v / ax[1]) ** 2 <= 1.0
        vol[inside] = rng.uniform(20.0, 220.0)
    coef = rng.normal(0.0, 0.5, size=6)
    w = zz / depth * 2.0 - 1.0
    uu = xx / (size - 1) * 2.0 - 1.0
    vv = yy / (size - 1) * 2.0 - 1.0
    bias = np.exp(0.3 * (coef[0] * uu + coef[1] * vv + coef[2] * uu * uu + coef[3] * vv * vv
                         + coef[4] * uu * vv + coef[5] * w))
    n1 = rng.normal(0.0, 4.0, size=vol.shape)
    n2 = rng.normal(0.0, 4.0, size=vol.shape)
    top = (1 << bits) - 1
    mag = np.sqrt((vol * bias + n1) ** 2 + n2 ** 2) * (top / 255.0)
    return np.clip(np.rint(mag), 0, top).astype(np.uint8 if bits == 8 else np.uint16)
