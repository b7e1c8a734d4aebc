"""12-bit samples on the GPU against the oracle: the 4096-output network's logits
against the oracle's BF16 form, tables against the oracle's FP32 rule over 64 blocks on
the GPU's own logits, streams byte for byte against the oracle's rANS of the GPU's
intervals (header with the depth marker), lossless round trips of images (several
encoder chunks included) and volumes through the four-phase cooperative decoder, the
256x256x35 12-bit scan at full size, and the error paths."""
import math

import numpy as np
import pytest
import torch

import oracle
import paper_2207_05152_amd as dl
import synth
from gpu_util import dev, say, to_dev  # noqa: F401
from oracle import softmax as sm
from oracle import volume as vo

pytestmark = pytest.mark.gpu
N = 4096


def _layers(H, seed, k_in=12, bias=0.05):
    layers = synth.xavier_deep(H, seed, k_in=k_in, n_out=N)
    rng = np.random.default_rng(seed + 1)
    return [(W, rng.normal(0, bias, b.shape).astype(np.float32)) for W, b in layers]


def _img(h, w, seed):
    return np.ascontiguousarray(synth.mri_volume(seed, 1, max(h, w), bits=12)[0][:h, :w])


def _d(a, dev):
    """12-bit samples live in int16 tensors on the device."""
    return to_dev(np.asarray(a).astype(np.int16), dev)


@pytest.fixture(scope="module", params=[64, 128])
def net(request, dev):
    H = request.param
    layers = _layers(H, 61 + H)
    return H, layers, dl.DeepModel(layers, dev)


def test_model_and_fingerprint(net):
    H, layers, m = net
    assert m.depth == 12 and m.fingerprint == sm.stored_fingerprint(layers)


def test_logits_match_oracle_bf16_form(dev, net):
    H, layers, m = net
    img = _img(23, 31, 5)
    say("d12 logits", H)
    lg, _, _ = dl.deep_density(_d(img, dev), m)
    torch.cuda.synchronize()
    got = lg.cpu().numpy().astype(np.float64)
    ref = sm.deep_forward_bf16(oracle.causal_features(img, 12).reshape(-1, 12), layers)
    err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
    assert err.max() <= 2.0 ** -6, err.max()
    per_px = err.max(axis=1)
    assert np.median(per_px) <= 1e-5, np.median(per_px)
    assert (per_px <= 2.0 ** -8).mean() >= 0.99


def test_tables_follow_the_fp32_rule(dev, net):
    H, layers, m = net
    img = _img(17, 21, 6)
    say("d12 tables", H)
    lg, cf, tab = dl.deep_density(_d(img, dev), m, tables=True)
    torch.cuda.synchronize()
    T = tab.cpu().numpy().view(np.uint16).astype(np.int64)
    F = np.concatenate([T, np.full((T.shape[0], 1), 65536)], axis=1)
    assert np.all(F[:, 0] == 0) and np.all(np.diff(F, axis=1) >= 1)
    ref = sm.table_softmax32(lg.cpu().numpy())
    d = np.abs(F - ref)
    assert d.max() <= 1 and (d == 0).mean() >= 0.999, (d.max(), (d == 0).mean())
    v = img.reshape(-1).astype(np.int64)
    rows = np.arange(v.size)
    c = cf.cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal(c & 0xFFFF, F[rows, v])
    assert np.array_equal((c >> 16) + 1, F[rows, v + 1] - F[rows, v])


@pytest.mark.parametrize("h,w,G,L", [(24, 30, 2, 4), (13, 50, 1, 16)])
def test_stream_is_oracle_rans_of_gpu_intervals(dev, net, h, w, G, L):
    H, layers, m = net
    img = _img(h, w, 7 + h)
    say("d12 stream", H, h, w, G, L)
    bits = dl.deep_encode(_d(img, dev), m, dl.dlic_coder(G, L))
    _, cf, _ = dl.deep_density(_d(img, dev), m, logits=False)
    torch.cuda.synchronize()
    c = cf.cpu().numpy().view(np.uint32).astype(np.int64)
    cc, ff = c & 0xFFFF, (c >> 16) + 1
    streams = []
    for grp in oracle.canonical_order(h, w, G, L):
        idx = [y * w + x for (y, x, _) in grp]
        streams.append(oracle.rans_encode([(cc[i], ff[i]) for i in idx], [t[2] for t in grp], L))
    hdr = oracle.pack_header(h, w, G, L, dtype=sm.header_dtype(12), h1=H, h2=H, n_mix=0,
                             fp=sm.stored_fingerprint(layers))
    assert bits.cpu().numpy().tobytes() == oracle.assemble(hdr, streams)


@pytest.mark.parametrize("h,w,G,L", [(24, 30, 2, 4), (40, 17, 1, 16), (9, 70, 3, 2), (1, 5, 1, 4),
                                     (160, 120, 4, 8)])
def test_round_trip(dev, net, h, w, G, L):
    # 160 x 120 = 19 200 pixels: the encoder runs two chunks of its stages
    H, layers, m = net
    img = _img(h, w, 100 + h + w)
    coder = dl.dlic_coder(G, L)
    say("d12 encode", H, h, w, G, L)
    bits = dl.deep_encode(_d(img, dev), m, coder)
    say("d12 decode", H, h, w, G, L)
    dec, st = dl.deep_decode(bits, m, check=False)
    torch.cuda.synchronize()
    assert st == 0
    assert np.array_equal(dec.cpu().numpy().astype(np.uint16), img)


@pytest.mark.parametrize("Z,h,w,G,L,ws", [(3, 20, 24, 2, 4, 0), (4, 17, 30, 1, 8, 1),
                                          (2, 33, 16, 3, 4, 2)])
def test_volume_round_trip(dev, net, Z, h, w, G, L, ws):
    H, _, _ = net
    layers = _layers(H, 5 + Z, k_in=21)
    m = dl.DeepModel(layers, dev)
    vol = synth.mri_volume(40 + Z, Z, max(h, w), bits=12)[:, :h, :w]
    say("d12 volume", H, Z, h, w, G, L, ws)
    bits = dl.volume_encode(_d(vol, dev), m, dl.dlic_coder(G, L), ws)
    dec, st = dl.volume_decode(bits, m, check=False)
    torch.cuda.synchronize()
    assert st == 0 and np.array_equal(dec.cpu().numpy().astype(np.uint16), vol)
    hdr = oracle.parse_header(bits[:oracle.HEADER_SIZE].cpu().numpy().tobytes())
    assert hdr["dtype"] == 0x41 and hdr["k_in"] == 21 and hdr["flags"] == vo.volume_flags(Z, ws)


def test_coded_length_near_ideal(dev, net):
    H, layers, m = net
    img = _img(40, 48, 9)
    bits = dl.deep_encode(_d(img, dev), m, dl.dlic_coder(1, 16))
    torch.cuda.synchronize()
    logits = sm.deep_forward_bf16(oracle.causal_features(img, 12).reshape(-1, 12), layers)
    ideal = sm.ideal_bits_softmax(logits, img.reshape(-1))
    payload = 8 * (bits.numel() - oracle.HEADER_SIZE - 4)
    # the 16-bit table's floor of one count per level costs at most -log2(15/16)
    assert ideal <= payload <= ideal + img.size * (-math.log2(15 / 16) + 0.02) + 32 * 16


def test_errors(dev, net):
    H, layers, m = net
    img = _img(20, 24, 3)
    coder = dl.dlic_coder(2, 4)
    bad = img.copy()
    bad[7, 9] = 4096
    say("d12 invalid sample")
    with pytest.raises(dl.DlicError):
        dl.deep_encode(_d(bad, dev), m, coder)
    bits = dl.deep_encode(_d(img, dev), m, coder)
    other = dl.DeepModel([(W, b + np.float32(0.01)) for W, b in layers], dev)
    say("d12 wrong model")
    _, st = dl.deep_decode(bits, other, check=False)
    assert st == dl.DLIC_ERR_MODEL_MISMATCH
    say("d12 truncated")
    _, st = dl.deep_decode(bits[:-2], m, check=False)
    assert st == dl.DLIC_ERR_CORRUPT
    # an 8-bit network of the same widths refuses the stream (the depth marker differs)
    m8 = dl.DeepModel(synth.xavier_deep(H, 61 + H), dev)
    bytes8 = torch.empty((20, 24), dtype=torch.uint8, device=dev)
    st8 = torch.zeros(1, dtype=torch.int32, device=dev)
    wsb = dl.dlic_deep_workspace(m8, 20, 24, coder, 1)
    wsp = torch.empty(wsb, dtype=torch.uint8, device=dev)
    rc = dl.lib().dlic_deep_decode(dl.ctypes.byref(m8.c), dl.ctypes.byref(coder), bits.data_ptr(),
                                   bits.numel(), bytes8.data_ptr(), 20, 24, st8.data_ptr(),
                                   wsp.data_ptr(), wsb, None)
    torch.cuda.synchronize()
    assert rc == 0 and int(st8.item()) == dl.DLIC_ERR_MODEL_MISMATCH
    with pytest.raises(ValueError):        # 8-bit samples for a 12-bit model
        dl.deep_encode(to_dev(img.astype(np.uint8), dev), m, coder)


def test_scan_full_size(dev):
    # a 12-bit 256x256x35 scan (the paper's MRI size and depth), 128-wide network,
    # window shift 1: round trip, and sampled logits against the oracle voxel by voxel
    layers = _layers(128, 77, k_in=21)
    m = dl.DeepModel(layers, dev)
    vol = synth.mri_volume(2024, bits=12)
    d_vol = _d(vol, dev)
    coder = dl.dlic_coder(8, 8)
    say("d12 full encode")
    bits = dl.volume_encode(d_vol, m, coder, 1)
    say("d12 full decode")
    dec, st = dl.volume_decode(bits, m, check=False)
    torch.cuda.synchronize()
    assert st == 0 and torch.equal(dec, d_vol)
    say("d12 full density, two slices")
    lg, _, _ = dl.volume_density(d_vol[:2].contiguous(), m, 1)
    rng = np.random.default_rng(5)
    idx = rng.integers(0, 2 * 256 * 256, 600)
    idx[:2] = [0, 2 * 256 * 256 - 1]
    got = lg[torch.from_numpy(idx).to(dev)].cpu().numpy().astype(np.float64)
    del lg
    zz, rem = np.divmod(idx, 256 * 256)
    yy, xx = np.divmod(rem, 256)
    feats = np.stack([vo.voxel_features(vol, z, y, x, 1, 12) for z, y, x in zip(zz, yy, xx)])
    ref = sm.deep_forward_bf16(feats, layers)
    err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
    assert err.max() <= 2.0 ** -6 and (err.max(axis=1) <= 2.0 ** -8).mean() >= 0.99
