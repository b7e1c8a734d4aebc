"""GPU encode -> GPU decode is lossless; stream structure and length agree with the oracle."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2207_05152_amd as dl
import synth
from gpu_util import dev, say, to_dev  # noqa: F401

pytestmark = pytest.mark.gpu


def _roundtrip(dev, img, wts, coder):
    m = dl.Model(wts, dev)
    d_img = to_dev(img, dev)
    say("encode", img.shape, coder.groups, coder.lanes_per_group)
    bits = dl.encode(d_img, m, coder)
    say("decode", img.shape, coder.groups, coder.lanes_per_group)
    dec, st = dl.decode(bits, m, check=False)
    torch.cuda.synchronize()
    return m, d_img, bits, dec.cpu().numpy(), st


@pytest.mark.parametrize("h,w,width,G,L", [
    (64, 64, 32, 1, 32), (1, 1, 32, 1, 32), (1, 9, 32, 1, 32), (9, 1, 64, 1, 32),
    (2, 3, 32, 1, 32), (5, 7, 64, 2, 4), (33, 4, 32, 2, 32), (100, 37, 64, 3, 32),
    (31, 70, 64, 1, 64), (50, 20, 32, 5, 3), (256, 256, 64, 2, 32), (96, 130, 64, 24, 4),
    (40, 50, 32, 8, 1), (37, 61, 128, 3, 2), (60, 90, 64, 10, 3)])
def test_lossless_round_trip(dev, h, w, width, G, L):
    img = synth.synth_image(h, w, 3 + h + w)
    wts = synth.xavier_mlp((12, width, width, 15), 3)
    _, _, bits, dec, st = _roundtrip(dev, img, wts, dl.dlic_coder(G, L))
    assert st == 0
    assert np.array_equal(dec, img)


def test_c0_stream_structure_and_rate(dev, c0_inputs):
    img, wts = c0_inputs
    m, d_img, bits, dec, st = _roundtrip(dev, img, wts, dl.dlic_coder(1, 32))
    assert st == 0 and np.array_equal(dec, img)
    raw = bits.cpu().numpy().tobytes()
    want_hdr = oracle.pack_header(64, 64, 1, 32, dtype=0, h1=32, h2=32,
                                  fp=oracle.weights_fingerprint(wts))
    assert raw[:36] == want_hdr
    # the encoder's stream is the rANS kernel applied to the density kernel's intervals
    _, cf, _ = dl.density(d_img, m)
    coder = dl.dlic_coder(1, 32)
    cap = dl.dlic_encode_bound(64, 64, coder)
    out = torch.zeros(cap, dtype=torch.uint8, device=dev)
    olen = torch.zeros(1, dtype=torch.int64, device=dev)
    wsb = dl.dlic_encode_workspace(64, 64, coder)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    dl.dlic_rans_encode_cf(coder, 64, 64, cf, out, cap, olen, ws, wsb)
    torch.cuda.synchronize()
    assert out[: int(olen.item())].cpu().numpy().tobytes()[36:] == raw[36:]
    # coded length: sum of -log2(f/M) of the GPU intervals, within the rANS
    # bounds, and that sum within log2(M/M') per pixel of the FP64 ideal
    cfn = cf.cpu().numpy().view(np.uint32).astype(np.int64)
    cost = math.fsum((-np.log2(((cfn >> 16) + 1) / 65536.0)).tolist())
    ideal = oracle.ideal_bits_image(img, wts)
    payload = 8 * (len(raw) - 36 - 4)
    assert cost <= ideal + img.size * (math.log2(65536 / 65280) + 1e-3)
    assert cost - 1 <= payload <= cost + 32 * 32 + 0.02 * img.size


# 8 x 32 and 64 x 4: 256 lanes; 384 x 4 and 48 x 32: one lane per row (one sub-round per step)
@pytest.mark.parametrize("G,L", [(8, 32), (64, 4), (384, 4), (48, 32)])
def test_full_size_round_trip(dev, G, L):
    img = synth.synth_image(1536, 2048, 1)
    wts = synth.xavier_mlp((12, 64, 64, 15), 3)
    _, _, bits, dec, st = _roundtrip(dev, img, wts, dl.dlic_coder(G, L))
    assert st == 0
    assert np.array_equal(dec, img)


def test_full_size_round_trip_width128(dev):
    # the 128-wide FP32 net at 64 groups x 4 lanes: the decoder's 4-pixel form
    # of layer 2 must reproduce the encoder's 16-pixel form bit for bit
    img = synth.synth_image(1536, 2048, 1)
    wts = synth.xavier_mlp((12, 128, 128, 15), 3)
    _, _, bits, dec, st = _roundtrip(dev, img, wts, dl.dlic_coder(64, 4))
    assert st == 0
    assert np.array_equal(dec, img)


def test_model_mismatch_and_corruption(dev, c0_inputs):
    img, wts = c0_inputs
    m, d_img, bits, dec, st = _roundtrip(dev, img, wts, dl.dlic_coder(1, 32))
    other = dict(wts)
    other["b3"] = wts["b3"] + np.float32(0.01)
    say("wrong model")
    _, st = dl.decode(bits, dl.Model(other, dev), check=False)
    assert st == dl.DLIC_ERR_MODEL_MISMATCH
    say("truncated stream")
    _, st = dl.decode(bits[:-2], m, check=False)
    assert st == dl.DLIC_ERR_CORRUPT
    bad = bits.clone()
    bad[bits.numel() // 2] ^= 0x33
    say("flipped byte")
    dec2, st = dl.decode(bad, m, check=False)
    torch.cuda.synchronize()
    assert st == dl.DLIC_ERR_CORRUPT or not np.array_equal(dec2.cpu().numpy(), img)
