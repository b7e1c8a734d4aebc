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


def test_c3_batch_against_oracle(dev):
    """Images from the batch workload (seeds 100-107, a 2048x1536 member among them), the
    12-64-64-15 net in BF16 and the layout the autotuner picks for them: every stream is the
    oracle's rANS of the batch's own intervals (byte for byte, header included), those
    intervals follow the oracle's BF16 network and FP32 table rule on sampled pixels of every
    image, and the decode is lossless."""
    from oracle import lowp
    import oracle
    from paper_2207_05152_amd import autotune
    seeds = list(range(100, 108))
    sizes = synth.batch_sizes(seeds)
    assert (1536, 2048) in sizes and (256, 256) in sizes
    imgs = [synth.synth_image(h, w, s) for (h, w), s in zip(sizes, seeds)]
    w = synth.xavier_mlp((12, 64, 64, 15), 3)
    model = dl.Model(w, dev, dtype="bf16")
    qm = lowp.quantize_weights(w, "bf16")
    assert model.fingerprint == lowp.stored_fingerprint(qm)
    say("c3 autotune")
    knobs = autotune.tune(model, sizes, imgs, reps=1, budget_s=20.0, use_cache=False)["knobs"]
    coders = autotune.coders_for(sizes, knobs["rows_per_group"], knobs["lanes"])
    say("c3 batch", knobs)
    b = dl.Batch(model, sizes, coders=coders, density_grid=knobs["density_grid"],
                 search_lanes=knobs["search_lanes"], decode_grid=knobs["decode_grid"])
    assert [tuple(c) for c in b.coders] == [tuple(c) for c in coders]
    b.load(imgs)
    b.capture()
    b.replay(decode=False)
    torch.cuda.synchronize()
    intervals = [b.intervals(i).cpu().numpy().view(np.uint32).astype(np.int64)
                 for i in range(len(sizes))]
    b.replay(decode=True)
    torch.cuda.synchronize()
    assert np.array_equal(b.status.cpu().numpy(), np.zeros(len(sizes)))
    rng = np.random.default_rng(1)
    for i, ((h, wd), img) in enumerate(zip(sizes, imgs)):
        assert np.array_equal(b.image(i).cpu().numpy(), img), i
        raw = b.stream(i).cpu().numpy().tobytes()
        G, L = (int(v) for v in coders[i])
        c = intervals[i] & 0xFFFF
        f = (intervals[i] >> 16) + 1
        assert (f >= 1).all() and (c + f <= 65536).all()
        # the stream is the oracle's coding of these intervals
        streams = []
        for grp in oracle.canonical_order(h, wd, G, L):
            ys = np.fromiter((t[0] for t in grp), np.int64, len(grp))
            xs = np.fromiter((t[1] for t in grp), np.int64, len(grp))
            ln = [t[2] for t in grp]
            streams.append(oracle.rans_encode(list(zip(c[ys, xs], f[ys, xs])), ln, L))
        hdr = oracle.pack_header(h, wd, G, L, dtype=dl.DLIC_BF16, h1=64, h2=64,
                                 fp=model.fingerprint)
        assert raw == oracle.assemble(hdr, streams), i
        # the intervals follow the oracle's BF16 network and FP32 table rule
        p = np.concatenate([rng.integers(0, h * wd, 400), [0, wd - 1, h * wd - wd, h * wd - 1]])
        ys, xs = p // wd, p % wd
        feats = np.stack([oracle.pixel_features(img, int(y), int(x)) for y, x in zip(ys, xs)])
        pi, mu, is_ = oracle.mixture_head(lowp.mlp_forward_lowp(feats, qm))
        v = img[ys, xs].astype(np.int64)
        F = oracle.table_levels32(np.stack([v, v + 1], 1), pi.astype(np.float32),
                                  mu.astype(np.float32), is_.astype(np.float32))
        dlo = np.abs(c[ys, xs] - F[:, 0])
        dhi = np.abs(c[ys, xs] + f[ys, xs] - F[:, 1])
        d = np.maximum(dlo, dhi)
        # GPU FP32 accumulation vs the oracle's exact sums: a count of 1 at a table
        # boundary; an activation at a BF16 tie can move more, rarely
        assert (d <= 1).mean() >= 0.99 and d.max() <= 512, (i, d.max())
        cost_gpu = -np.log2(f[ys, xs] / 65536.0).mean()
        cost_ora = -np.log2((F[:, 1] - F[:, 0]) / 65536.0).mean()
        assert abs(cost_gpu - cost_ora) <= 1e-3, i
    b.close()


def test_batch_decode_knobs_do_not_change_results(dev):
    model = dl.Model(synth.xavier_mlp((12, 64, 64, 15), 3), dev, dtype="bf16")
    sizes = [(96, 130), (40, 56), (130, 70), (17, 200)]
    imgs = _images(sizes, 900)
    coders = [(max(1, h // 12), 4) for h, _ in sizes]
    ref = None
    for search, grid in ((0, 0), (2, 0), (1, 3), (16, 1)):
        say("batch knobs", search, grid)
        b = dl.Batch(model, sizes, coders=coders, search_lanes=search, decode_grid=grid)
        b.load(imgs)
        b.encode()
        b.decode()
        torch.cuda.synchronize()
        assert np.array_equal(b.status.cpu().numpy(), np.zeros(len(sizes)))
        streams = [b.stream(i).cpu().numpy() for i in range(len(sizes))]
        for i, img in enumerate(imgs):
            assert np.array_equal(b.image(i).cpu().numpy(), img), (search, grid, i)
        if ref is None:
            ref = streams
        for a, r in zip(streams, ref):
            assert np.array_equal(a, r)
        b.close()
    # 16 lanes per pixel need layouts of at most 4 lanes
    with pytest.raises(dl.DlicError):
        dl.Batch(model, [(64, 64)], coders=[(2, 32)], search_lanes=16)
    with pytest.raises(dl.DlicError):
        dl.Batch(model, [(64, 64)], coders=[(2, 64)], search_lanes=2)
