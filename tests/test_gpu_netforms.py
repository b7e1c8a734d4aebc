"""The two FP32 forms of the 12-H-H-15 network (H = 64, 128), on the GPU through the C-ABI test hook:
the encoder's 16-pixel tiles (16x16x4 MFMA) and the decoder's 4-pixel tiles (4x4x1 MFMA),
bit for bit on the same features, and both against a CPU statement of the summation order
they share: every output a chain of correctly rounded FP32 fused multiply-adds, layer by
layer in a fixed input order, layer 3 in four quarters added ((q0 + q1) + q2) + q3."""
import numpy as np
import pytest
import torch

import paper_2207_05152_amd as dl
import synth
from gpu_util import dev, say, to_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def fma32(a, b, c):
    """Correctly rounded FP32 a * b + c, elementwise (exact product in FP64, exact sum by
    TwoSum, then one rounding to FP32 that resolves FP64 ties at FP32 midpoints)."""
    a64, b64, c64 = (np.asarray(x, np.float32).astype(np.float64) for x in (a, b, c))
    p = a64 * b64
    s = p + c64
    bb = s - p
    e = (p - (s - bb)) + (c64 - bb)
    r = s.astype(np.float32)
    r64 = r.astype(np.float64)
    d = s - r64
    up = np.nextafter(r, np.float32(np.inf))
    dn = np.nextafter(r, np.float32(-np.inf))
    mid_hi = d == (up.astype(np.float64) - r64) / 2
    mid_lo = d == -(r64 - dn.astype(np.float64)) / 2
    r = np.where(mid_hi & (d != 0) & (e > 0), up, r)
    r = np.where(mid_lo & (d != 0) & (e < 0), dn, r)
    return r


def test_fma32_emulation_cases():
    f = np.float32
    one = f(1.0)
    eps = np.float32(2.0 ** -23)
    # 1 + 2^-24 is a tie in FP32: an exact product term decides it
    assert fma32(f(2.0 ** -12), f(2.0 ** -12), one) == one
    assert fma32(f(2.0 ** -12), f(2.0 ** -12 * (1 + 2.0 ** -20)), one) == one + eps
    assert fma32(f(-(2.0 ** -12)), f(2.0 ** -12 * (1 + 2.0 ** -20)), one + eps) == one
    # a product whose low bits a separate multiply would lose
    x = f(1 + 2.0 ** -12)
    assert fma32(x, x, f(-1.0)) == f(2.0 ** -11 + 2.0 ** -24)
    assert (np.float32(x * x) - f(1.0)) == f(2.0 ** -11)


def kc(c):   # input of layer-2 chain step c
    return 16 * (c // 16) + 4 * (c % 4) + (c % 16) // 4


def k3(g, st, H=128):   # input of step st of layer-3 quarter g (H / 4 steps per quarter)
    return 16 * ((H // 64) * g + (st >> 4)) + 4 * (st & 3) + ((st >> 2) & 3)


def net_chain32(f, w):
    """12-H-H-15 FP32 in the shared order, every step one correctly rounded FMA."""
    f = f.astype(np.float32)
    W1, W2, W3 = (w[k].astype(np.float32) for k in ("W1", "W2", "W3"))
    H = W1.shape[0]
    acc = np.broadcast_to(w["b1"].astype(np.float32), (f.shape[0], H)).copy()
    for k in range(12):
        acc = fma32(W1[None, :, k], f[:, k:k + 1], acc)
    h1 = np.where(acc > 0, acc, np.float32(0))
    acc = np.broadcast_to(w["b2"].astype(np.float32), (f.shape[0], H)).copy()
    for c in range(H):
        k = kc(c)
        acc = fma32(W2[None, :, k], h1[:, k:k + 1], acc)
    h2 = np.where(acc > 0, acc, np.float32(0))
    quarters = []
    for g in range(4):
        q = np.broadcast_to(w["b3"].astype(np.float32) if g == 0 else np.zeros(15, np.float32),
                            (f.shape[0], 15)).copy()
        for st in range(H // 4):
            k = k3(g, st, H)
            q = fma32(W3[None, :, k], h2[:, k:k + 1], q)
        quarters.append(q)
    return ((quarters[0] + quarters[1]) + quarters[2]) + quarters[3]


@pytest.mark.parametrize("H", [64, 128])
def test_layer_orders_are_permutations(H):
    assert sorted(kc(c) for c in range(H)) == list(range(H))
    assert sorted(k3(g, s, H) for g in range(4) for s in range(H // 4)) == list(range(H))


def _features(n, seed):
    rng = np.random.default_rng(seed)
    f = rng.uniform(-1, 1, (n, 12))
    kind = rng.integers(0, 5, n)
    f[kind == 1] = (2.0 * rng.integers(0, 256, (int((kind == 1).sum()), 12)) - 255) / 255
    f[kind == 2] *= 8.0                                    # wide magnitudes
    f[kind == 3] *= 1e-6                                   # tiny inputs
    half = f[kind == 4]
    half[:, 6:] = -half[:, :6]                             # cancelling pairs
    f[kind == 4] = half
    f[rng.random((n, 12)) < 0.1] = 0.0                     # dummy neighbours
    return f.astype(np.float32)


def _weights(seed, scale, H=128):
    w = synth.xavier_mlp((12, H, H, 15), seed)
    rng = np.random.default_rng(seed + 1)
    for k in ("W1", "W2", "W3"):
        w[k] = (w[k] * scale).astype(np.float32)
    for k in ("b1", "b2", "b3"):
        w[k] = rng.normal(0, 0.3, w[k].shape).astype(np.float32)
    return w


@pytest.mark.parametrize("H,seed,scale", [(128, 3, 1.0), (128, 11, 4.0), (64, 3, 1.0),
                                          (64, 11, 4.0)])
def test_four_pixel_form_equals_sixteen_pixel_form(dev, H, seed, scale):
    w = _weights(seed, scale, H)
    m = dl.Model(w, dev)
    n = 4096
    feats = _features(n, seed)
    d_f = to_dev(feats, dev)
    o16 = torch.empty((n, 15), dtype=torch.float32, device=dev)
    o4 = torch.empty((n, 15), dtype=torch.float32, device=dev)
    for lanes in (4, 3, 2, 1):
        say("net forms", H, seed, scale, lanes)
        o4.fill_(float("nan"))
        dl.dlic_net_forms(m.c, d_f, n, lanes, o16, o4)
        torch.cuda.synchronize()
        a = o16.cpu().numpy()
        b = o4.cpu().numpy()
        rows = (np.arange(n) % 4) < lanes
        assert np.array_equal(a[rows].view(np.uint32), b[rows].view(np.uint32)), lanes
    # both are the correctly rounded FMA chain in the shared order
    ref = net_chain32(feats[:256], w)
    assert np.array_equal(a[:256], ref), np.abs(a[:256] - ref).max()


def test_net_forms_rejects_other_models(dev):
    m = dl.Model(synth.xavier_mlp((12, 32, 32, 15), 3), dev)
    x = torch.zeros((16, 15), dtype=torch.float32, device=dev)
    with pytest.raises(dl.DlicError):
        dl.dlic_net_forms(m.c, x, 16, 4, x, x)
