"""Density parity: GPU network outputs vs the FP64 oracle, GPU tables vs the
oracle's FP32 table rule (the kernel's precision for the integer decision)."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2207_05152_amd as dl
import synth
from gpu_util import dev, say, to_dev  # noqa: F401

pytestmark = pytest.mark.gpu

TOL = 1e-4   # |gpu - ref| <= TOL * max(1, |ref|) for every network output


def _oracle_out(img, w, idx=None):
    if idx is None:
        feats = oracle.causal_features(img)
    else:
        feats = np.stack([oracle.pixel_features(img, int(p) // img.shape[1], int(p) % img.shape[1])
                          for p in idx])
    return oracle.mlp_forward(feats, w["W1"], w["b1"], w["W2"], w["b2"], w["W3"], w["b3"])


def _rel_err(gpu, ref):
    return np.abs(gpu.astype(np.float64) - ref) / np.maximum(1.0, np.abs(ref))


@pytest.mark.parametrize("h,w,width,seed", [(64, 64, 32, 7), (37, 53, 64, 3), (3, 2, 32, 5),
                                            (1, 17, 64, 3)])
def test_outputs_match_fp64_oracle(dev, h, w, width, seed):
    img = synth.synth_image(h, w, 42 + h)
    wts = synth.xavier_mlp((12, width, width, 15), seed)
    wts["b1"] = np.linspace(-0.1, 0.1, width).astype(np.float32)
    wts["b3"] = np.linspace(-0.5, 0.5, 15).astype(np.float32)
    m = dl.Model(wts, dev)
    say("density", h, w, width)
    out15, cf, _ = dl.density(to_dev(img, dev), m)
    torch.cuda.synchronize()
    err = _rel_err(out15.cpu().numpy(), _oracle_out(img, wts))
    assert err.max() <= TOL, err.max()


def test_full_size_outputs_sampled(dev):
    img = synth.synth_image(1536, 2048, 1)
    wts = synth.xavier_mlp((12, 64, 64, 15), 3)
    m = dl.Model(wts, dev)
    say("density full size")
    out15, _, _ = dl.density(to_dev(img, dev), m)
    torch.cuda.synchronize()
    rng = np.random.default_rng(0)
    idx = np.concatenate([rng.integers(0, img.size, 3000), [0, 1, 2047, 2048, img.size - 1]])
    err = _rel_err(out15.cpu().numpy()[idx], _oracle_out(img, wts, idx))
    assert err.max() <= TOL, err.max()


def test_position_in_tile_does_not_change_bits(dev):
    # Prepending a column shifts every pixel's raster index (and so its
    # position inside a 16-pixel tile) while windows with x >= 2 stay equal.
    img = synth.synth_image(40, 61, 9)
    wide = np.concatenate([synth.synth_image(40, 1, 10), img], axis=1)
    m = dl.Model(synth.xavier_mlp((12, 64, 64, 15), 3), dev)
    say("tile position invariance")
    a, ca, _ = dl.density(to_dev(img, dev), m)
    b, cb, _ = dl.density(to_dev(wide, dev), m)
    torch.cuda.synchronize()
    a = a.cpu().numpy().reshape(40, 61, 15)[:, 2:]
    b = b.cpu().numpy().reshape(40, 62, 15)[:, 3:]
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
    ca = ca.cpu().numpy().reshape(40, 61)[:, 2:]
    cb = cb.cpu().numpy().reshape(40, 62)[:, 3:]
    assert np.array_equal(ca, cb)


def test_tables_valid_and_match_oracle_rule(dev):
    h, w = 24, 40
    img = synth.synth_image(h, w, 11)
    wts = synth.xavier_mlp((12, 32, 32, 15), 7)
    m = dl.Model(wts, dev)
    say("tables", h, w)
    out15, cf, tab = dl.density(to_dev(img, dev), m, tables=True)
    torch.cuda.synchronize()
    tg = tab.cpu().numpy().astype(np.int64)
    f = np.diff(tg, axis=1)
    assert (tg[:, 0] == 0).all() and (tg[:, -1] == 65536).all() and (f >= 1).all()
    # the packed interval of each pixel is read off its own table
    v = img.ravel().astype(np.int64)
    cfg = cf.cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal(cfg & 0xFFFF, tg[np.arange(h * w), v])
    assert np.array_equal((cfg >> 16) + 1, tg[np.arange(h * w), v + 1] - tg[np.arange(h * w), v])
    # oracle: FP64 network, parameters rounded to FP32, FP32 table rule
    o64 = _oracle_out(img, wts)
    pi, mu, is_ = oracle.mixture_head(o64)
    to = oracle.table_full32(pi.astype(np.float32), mu.astype(np.float32), is_.astype(np.float32))
    d = tg - to
    assert np.abs(d).max() <= 1
    # where the two differ, the oracle's pre-floor value must lie within the
    # error the measured output differences can propagate to it
    og = out15.cpu().numpy().astype(np.float64)
    da = np.abs(og[:, 0:5] - o64[:, 0:5]).max(axis=1)
    dmu = np.abs(og[:, 5:10] - o64[:, 5:10])
    dls = np.abs(og[:, 10:15] - o64[:, 10:15])
    beta = oracle.beta32().astype(np.float64)
    S, D = oracle.sigma_lut32()
    pp, vv = np.nonzero(d)
    for p, lv in zip(pp, vv):
        b = beta[lv]
        t = (b - mu[p]) * is_[p]
        z = 65280.0 * float(np.sum(pi[p] * (1.0 / (1.0 + np.exp(-t)))))
        dz = 65280.0 * float(np.sum(2 * pi[p] * da[p] + pi[p] * 0.25 *
                                    (dmu[p] * is_[p] + np.abs(b - mu[p]) * is_[p] * dls[p])) + 2e-6)
        assert abs(z - round(z)) <= 4 * dz + 0.06, (p, lv, z, dz)
    assert d.astype(bool).mean() < 0.05
    # cost of coding the image with either table set differs negligibly
    cost = lambda T: float(np.sum(-np.log2((T[np.arange(h * w), v + 1] - T[np.arange(h * w), v]) / 65536.0)))
    assert abs(cost(tg) - cost(to)) / (h * w) <= 1e-3
