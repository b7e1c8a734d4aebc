"""Batched encode/decode of uneven images in one launch per direction, and
its hipGraph capture: every image's stream must be the bytes the
single-image path writes for it (whose parity with the oracle the other GPU
tests establish), every decode lossless, every replay equal to eager work."""
import numpy as np
import pytest
import torch

import paper_2207_05152_amd as dl
import synth
from gpu_util import dev, say, to_dev  # noqa: F401

pytestmark = pytest.mark.gpu

SIZES = [(40, 56), (64, 64), (23, 100), (100, 30), (8, 200), (130, 70), (2, 9), (200, 17)]


def _images(sizes, base):
    return [synth.synth_image(h, w, base + i) for i, (h, w) in enumerate(sizes)]


def _single(img, model, coder, dev):
    return dl.encode(to_dev(img, dev), model, coder).cpu().numpy()


@pytest.mark.parametrize("dtype,width", [("fp32", 64), ("bf16", 64), ("fp8", 32), ("bf16", 128)])
def test_batch_streams_equal_single_image_streams(dev, dtype, width):
    model = dl.Model(synth.xavier_mlp((12, width, width, 15), 3), dev, dtype=dtype)
    coders = [(max(1, min(h // 24, 4)), 32 if i % 2 else 16) for i, (h, w) in enumerate(SIZES)]
    imgs = _images(SIZES, 300)
    say("batch eager", dtype, width, len(SIZES))
    b = dl.Batch(model, SIZES, coders=coders)
    b.load(imgs)
    b.encode()
    b.decode()
    torch.cuda.synchronize()
    assert np.array_equal(b.status.cpu().numpy(), np.zeros(len(SIZES)))
    for i, img in enumerate(imgs):
        want = _single(img, model, dl.dlic_coder(*coders[i]), dev)
        got = b.stream(i).cpu().numpy()
        assert np.array_equal(got, want), i
        assert np.array_equal(b.image(i).cpu().numpy(), img), i
    b.close()


@pytest.mark.parametrize("dtype,width", [("fp32", 64), ("bf16", 64), ("fp32", 32), ("fp32", 128)])
def test_batch_small_lane_layouts(dev, dtype, width):
    # 1 to 4 lanes per group: the decoder's coder gives each pixel 16 lanes
    model = dl.Model(synth.xavier_mlp((12, width, width, 15), 5), dev, dtype=dtype)
    coders = [(max(1, min(h // 8, 6)), 1 + i % 4) for i, (h, w) in enumerate(SIZES)]
    imgs = _images(SIZES, 700)
    say("batch small lanes", dtype, width)
    b = dl.Batch(model, SIZES, coders=coders)
    b.load(imgs)
    b.encode()
    b.decode()
    torch.cuda.synchronize()
    assert np.array_equal(b.status.cpu().numpy(), np.zeros(len(SIZES)))
    for i, img in enumerate(imgs):
        want = _single(img, model, dl.dlic_coder(*coders[i]), dev)
        assert np.array_equal(b.stream(i).cpu().numpy(), want), i
        assert np.array_equal(b.image(i).cpu().numpy(), img), i
    b.close()


def test_batch_default_layout_and_work_order(dev):
    model = dl.Model(synth.xavier_mlp((12, 32, 32, 15), 7), dev)
    sizes = [(300, 40), (16, 16), (193, 20), (385, 12)]
    b = dl.Batch(model, sizes)
    # default layout: ceil(h / 192) groups of 32 lanes
    assert [tuple(c) for c in b.coders] == [(2, 32), (1, 32), (2, 32), (3, 32)]
    assert b.n_items == 8
    imgs = _images(sizes, 50)
    say("batch default layout")
    b.load(imgs)
    b.encode()
    b.decode()
    torch.cuda.synchronize()
    for i, img in enumerate(imgs):
        assert np.array_equal(b.image(i).cpu().numpy(), img)
    lat = b.latencies_s(decode=True)
    assert np.all(lat > 0) and np.all(lat < 10), lat
    b.close()


def test_graph_replays_match_eager(dev):
    model = dl.Model(synth.xavier_mlp((12, 64, 64, 15), 3), dev, dtype="bf16")
    b = dl.Batch(model, SIZES)
    first = _images(SIZES, 400)
    second = _images(SIZES, 500)
    b.load(first)
    say("graph capture")
    b.capture()
    for rep, imgs in enumerate([first, second, first]):
        b.load(imgs)
        # eager work between replays: the single-image path on its own buffers
        want = [_single(im, model, dl.dlic_coder(*b.coders[i]), dev) for i, im in enumerate(imgs)]
        b.decoded.zero_()
        say("graph replay", rep)
        b.replay(decode=False)
        torch.cuda.synchronize()
        b.replay(decode=True)
        torch.cuda.synchronize()
        assert np.array_equal(b.status.cpu().numpy(), np.zeros(len(SIZES))), rep
        for i, im in enumerate(imgs):
            assert np.array_equal(b.stream(i).cpu().numpy(), want[i]), (rep, i)
            assert np.array_equal(b.image(i).cpu().numpy(), im), (rep, i)
        assert np.all(b.latencies_s(decode=False) > 0)
    b.close()


def test_batch_corrupt_image_is_isolated(dev):
    model = dl.Model(synth.xavier_mlp((12, 32, 32, 15), 7), dev)
    sizes = [(64, 80), (50, 50), (90, 33)]
    imgs = _images(sizes, 70)
    b = dl.Batch(model, sizes, coders=[(2, 32), (2, 32), (3, 16)])
    b.load(imgs)
    b.encode()
    torch.cuda.synchronize()
    o = int(b.out_off[1])
    b.out[o + 8] ^= 0xFF            # image 1: height field of the header
    b.lens[2] = 1 << 40             # image 2: length beyond its region
    say("batch corrupt isolation")
    b.decode()
    torch.cuda.synchronize()
    st = b.status.cpu().numpy()
    assert st[0] == dl.DLIC_OK and st[1] == dl.DLIC_ERR_CORRUPT and st[2] == dl.DLIC_ERR_CORRUPT
    assert np.array_equal(b.image(0).cpu().numpy(), imgs[0])
    b.close()


def test_batch_rejects_bad_plans(dev):
    model = dl.Model(synth.xavier_mlp((12, 32, 32, 15), 7), dev)
    with pytest.raises(dl.DlicError):
        dl.Batch(model, [(10, 10), (0, 5)])
    with pytest.raises(dl.DlicError):
        dl.Batch(model, [(600, 10)], coders=[(2, 32)])   # 300 rows per group
    with pytest.raises(dl.DlicError):
        dl.Batch(model, [(10, 10)], coders=[(1, 65)])
