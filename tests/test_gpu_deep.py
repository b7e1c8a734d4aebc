"""The paper's six-layer softmax-256 network on the GPU against the oracle: logits against
the oracle's BF16 form of the network, tables against the oracle's FP32 table rule applied
to the GPU's own logits, streams byte for byte against the oracle's rANS of the GPU's
intervals (header included), lossless round trips through the cooperative per-step
decoder, and the coded length against the ideal length."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2207_05152_amd as dl
import synth
from gpu_util import dev, say, to_dev  # noqa: F401
from oracle import softmax as sm

pytestmark = pytest.mark.gpu


def _layers(H, seed, bias=0.05):
    layers = synth.xavier_deep(H, seed)
    rng = np.random.default_rng(seed + 1)
    return [(W, rng.normal(0, bias, b.shape).astype(np.float32)) for W, b in layers]


@pytest.fixture(scope="module", params=[64, 128])
def net(request, dev):
    H = request.param
    layers = _layers(H, 11 + H)
    return H, layers, dl.DeepModel(layers, dev)


def test_fingerprint_is_the_oracles(net):
    H, layers, m = net
    assert m.fingerprint == sm.stored_fingerprint(layers)


def test_logits_match_oracle_bf16_form(dev, net):
    H, layers, m = net
    img = synth.synth_image(37, 53, 5)
    say("deep logits", H)
    lg, _, _ = dl.deep_density(to_dev(img, dev), m)
    torch.cuda.synchronize()
    got = lg.cpu().numpy().astype(np.float64)
    ref = sm.deep_forward_bf16(oracle.causal_features(img).reshape(-1, 12), layers)
    err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
    # FP32 accumulation (the oracle sums exactly) and, rarely, a hidden activation on the
    # other side of a BF16 tie: one BF16 step of one activation moves a logit by far less
    # than 2^-6 of its size; most pixels agree to FP32 accumulation accuracy
    assert err.max() <= 2.0 ** -6, err.max()
    per_px = err.max(axis=1)
    assert np.median(per_px) <= 1e-5, np.median(per_px)
    assert (per_px <= 2.0 ** -8).mean() >= 0.99


def test_tables_follow_the_fp32_rule(dev, net):
    H, layers, m = net
    img = synth.synth_image(29, 41, 6)
    say("deep tables", H)
    lg, cf, tab = dl.deep_density(to_dev(img, dev), m, tables=True)
    torch.cuda.synchronize()
    T = tab.cpu().numpy().view(np.uint16).astype(np.int64)
    F = np.concatenate([T, np.full((T.shape[0], 1), 65536)], axis=1)
    assert np.all(F[:, 0] == 0) and np.all(np.diff(F, axis=1) >= 1)
    # the oracle's rule on the GPU's own logits: equal but where expf and the exactly
    # rounded exponential differ by an ulp, which moves a count by at most one
    ref = sm.table_softmax32(lg.cpu().numpy())
    d = np.abs(F - ref)
    assert d.max() <= 1 and (d == 0).mean() >= 0.999, (d.max(), (d == 0).mean())
    # the intervals are the tables at each pixel's own level
    v = img.reshape(-1).astype(np.int64)
    rows = np.arange(v.size)
    c = cf.cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal(c & 0xFFFF, F[rows, v])
    assert np.array_equal((c >> 16) + 1, F[rows, v + 1] - F[rows, v])


@pytest.mark.parametrize("h,w,G,L", [(40, 56, 2, 4), (33, 70, 1, 32)])
def test_stream_is_oracle_rans_of_gpu_intervals(dev, net, h, w, G, L):
    H, layers, m = net
    img = synth.synth_image(h, w, 7 + h)
    coder = dl.dlic_coder(G, L)
    say("deep stream", H, h, w, G, L)
    bits = dl.deep_encode(to_dev(img, dev), m, coder)
    _, cf, _ = dl.deep_density(to_dev(img, dev), m, logits=False)
    torch.cuda.synchronize()
    c = cf.cpu().numpy().view(np.uint32).astype(np.int64)
    cc, ff = c & 0xFFFF, (c >> 16) + 1
    streams = []
    for grp in oracle.canonical_order(h, w, G, L):
        idx = [y * w + x for (y, x, _) in grp]
        streams.append(oracle.rans_encode([(cc[i], ff[i]) for i in idx], [t[2] for t in grp], L))
    hdr = oracle.pack_header(h, w, G, L, dtype=1, h1=H, h2=H, n_mix=0,
                             fp=sm.stored_fingerprint(layers))
    assert bits.cpu().numpy().tobytes() == oracle.assemble(hdr, streams)


@pytest.mark.parametrize("h,w,G,L", [(48, 64, 4, 4), (20, 33, 1, 32), (70, 25, 3, 8),
                                     (9, 130, 2, 64), (1, 5, 1, 4), (64, 64, 16, 4)])
def test_round_trip(dev, net, h, w, G, L):
    H, layers, m = net
    img = synth.synth_image(h, w, 100 + h + w)
    coder = dl.dlic_coder(G, L)
    say("deep encode", H, h, w, G, L)
    bits = dl.deep_encode(to_dev(img, dev), m, coder)
    say("deep decode", H, h, w, G, L)
    dec, st = dl.deep_decode(bits, m, check=False)
    torch.cuda.synchronize()
    assert st == 0
    assert np.array_equal(dec.cpu().numpy(), img)


def test_coded_length_near_ideal(dev, net):
    H, layers, m = net
    h, w = 48, 96
    img = synth.synth_image(h, w, 9)
    bits = dl.deep_encode(to_dev(img, dev), m, dl.dlic_coder(1, 32))
    torch.cuda.synchronize()
    logits = sm.deep_forward_bf16(oracle.causal_features(img).reshape(-1, 12), layers)
    ideal = sm.ideal_bits_softmax(logits, img.reshape(-1))
    payload = 8 * (bits.numel() - oracle.HEADER_SIZE - 4)
    assert payload <= ideal + img.size * (math.log2(65536 / 65280) + 0.02) + 32 * 32


def test_wrong_model_and_corruption(dev, net):
    H, layers, m = net
    img = synth.synth_image(24, 30, 3)
    coder = dl.dlic_coder(2, 4)
    bits = dl.deep_encode(to_dev(img, dev), m, coder)
    other = dl.DeepModel([(W, b + np.float32(0.01)) for W, b in layers], dev)
    say("deep wrong model")
    _, st = dl.deep_decode(bits, other, check=False)
    assert st == dl.DLIC_ERR_MODEL_MISMATCH
    say("deep truncated")
    _, st = dl.deep_decode(bits[:-2], m, check=False)
    assert st == dl.DLIC_ERR_CORRUPT
    # the mixture decoder refuses a softmax stream
    mix = dl.Model(synth.xavier_mlp((12, 64, 64, 15), 3), dev)
    _, st = dl.decode(bits, mix, check=False)
    assert st != 0
