"""Volumes on the GPU against the oracle: the 3-D window's logits against the oracle's
BF16 network on its 21 window values, tables against the oracle's FP32 table rule on the
GPU's own logits, streams byte for byte against the oracle's rANS of the GPU's intervals
(header with the slice count and window shift included), lossless round trips through the
3-D wavefront decoder for every window shift the tests name, ragged and degenerate shapes,
a forced small grid, the 256x256x35 scan at full size, and the error paths."""
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


def _layers(H, seed, k_in=21, bias=0.05):
    layers = synth.xavier_deep(H, seed, k_in=k_in)
    rng = np.random.default_rng(seed + 1)
    return [(W, rng.normal(0, bias, b.shape).astype(np.float32)) for W, b in layers]


@pytest.fixture(scope="module", params=[64, 128])
def net(request, dev):
    H = request.param
    layers = _layers(H, 41 + H)
    return H, layers, dl.DeepModel(layers, dev)


def _vol(Z, h, w, seed):
    v = synth.mri_volume(seed, depth=Z, size=max(h, w))
    return np.ascontiguousarray(v[:, :h, :w])


@pytest.mark.parametrize("ws", [0, 1, 2])
def test_logits_match_oracle_bf16_form(dev, net, ws):
    H, layers, m = net
    vol = _vol(3, 23, 29, 5 + ws)
    say("volume logits", H, ws)
    lg, _, _ = dl.volume_density(to_dev(vol, dev), m, ws)
    torch.cuda.synchronize()
    got = lg.cpu().numpy().astype(np.float64)
    ref = sm.deep_forward_bf16(vo.volume_features(vol, ws).reshape(-1, 21), layers)
    err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
    # as for images: FP32 accumulation against exact sums, rarely one BF16 tie of a
    # hidden activation
    assert err.max() <= 2.0 ** -6, err.max()
    per_px = err.max(axis=1)
    assert np.median(per_px) <= 1e-5, np.median(per_px)
    assert (per_px <= 2.0 ** -8).mean() >= 0.99


def test_lower_window_moves_the_logits(dev, net):
    # the same slice above two different slices: only the lower window differs
    H, layers, m = net
    a = _vol(2, 16, 16, 1)
    b = a.copy()
    b[0] = 255 - b[0]
    la, _, _ = dl.volume_density(to_dev(a, dev), m, 1)
    lb, _, _ = dl.volume_density(to_dev(b, dev), m, 1)
    torch.cuda.synchronize()
    n = 16 * 16
    da = np.abs(la[n:].cpu().numpy() - lb[n:].cpu().numpy()).max(axis=1)
    assert (da > 0).mean() > 0.9
    # with ws = 1 the window of row 0 still holds row 0 of the slice below
    ref_a = sm.deep_forward_bf16(vo.volume_features(a, 1).reshape(-1, 21), layers)[n:]
    ref_b = sm.deep_forward_bf16(vo.volume_features(b, 1).reshape(-1, 21), layers)[n:]
    assert np.all((np.abs(ref_a - ref_b).max(axis=1) > 0) == (da > 0))


def test_tables_follow_the_fp32_rule(dev, net):
    H, layers, m = net
    vol = _vol(2, 19, 21, 8)
    say("volume tables", H)
    lg, cf, tab = dl.volume_density(to_dev(vol, dev), m, 2, tables=True)
    torch.cuda.synchronize()
    T = tab.cpu().numpy().view(np.uint16).astype(np.int64)
    F = np.concatenate([T, np.full((T.shape[0], 1), 65536)], axis=1)
    assert np.all(F[:, 0] == 0) and np.all(np.diff(F, axis=1) >= 1)
    ref = sm.table_softmax32(lg.cpu().numpy())
    d = np.abs(F - ref)
    assert d.max() <= 1 and (d == 0).mean() >= 0.999, (d.max(), (d == 0).mean())
    v = vol.reshape(-1).astype(np.int64)
    rows = np.arange(v.size)
    c = cf.cpu().numpy().view(np.uint32).astype(np.int64)
    assert np.array_equal(c & 0xFFFF, F[rows, v])
    assert np.array_equal((c >> 16) + 1, F[rows, v + 1] - F[rows, v])


@pytest.mark.parametrize("Z,h,w,G,L,ws", [(3, 20, 24, 2, 4, 1), (2, 33, 17, 3, 8, 0),
                                          (4, 9, 40, 1, 16, 3)])
def test_stream_is_oracle_rans_of_gpu_intervals(dev, net, Z, h, w, G, L, ws):
    H, layers, m = net
    vol = _vol(Z, h, w, 17 + h)
    say("volume stream", H, Z, h, w, G, L, ws)
    bits = dl.volume_encode(to_dev(vol, dev), m, dl.dlic_coder(G, L), ws)
    _, cf, _ = dl.volume_density(to_dev(vol, dev), m, ws, logits=False)
    torch.cuda.synchronize()
    c = cf.cpu().numpy().view(np.uint32).astype(np.int64)
    cc, ff = c & 0xFFFF, (c >> 16) + 1
    streams = []
    for grp in oracle.canonical_order(Z * h, w, Z * G, L):
        idx = [y * w + x for (y, x, _) in grp]
        streams.append(oracle.rans_encode([(cc[i], ff[i]) for i in idx], [t[2] for t in grp], L))
    hdr = oracle.pack_header(Z * h, w, Z * G, L, dtype=1, h1=H, h2=H, n_mix=0, k_in=21,
                             fp=sm.stored_fingerprint(layers), flags=vo.volume_flags(Z, ws))
    assert bits.cpu().numpy().tobytes() == oracle.assemble(hdr, streams)
    hv = dl.dlic_peek_volume(bits[:oracle.HEADER_SIZE].cpu().numpy().tobytes())
    assert (hv["z"], hv["h"], hv["ws"], hv["k_in"]) == (Z, h, ws, 21)
    assert (hv["coder"].groups, hv["coder"].lanes_per_group) == (G, L)


@pytest.mark.parametrize("Z,h,w,G,L,ws", [
    (3, 20, 24, 2, 4, 0), (4, 17, 30, 1, 8, 1), (2, 33, 16, 3, 4, 2), (5, 9, 40, 1, 16, 3),
    (1, 12, 12, 1, 4, 1), (64, 8, 10, 1, 4, 1), (3, 10, 10, 1, 4, 15), (2, 5, 1, 1, 4, 1),
    (6, 40, 3, 2, 2, 2)])
def test_round_trip(dev, net, Z, h, w, G, L, ws):
    H, layers, m = net
    vol = _vol(Z, h, w, 100 + Z + h + w)
    coder = dl.dlic_coder(G, L)
    say("volume encode", H, Z, h, w, G, L, ws)
    bits = dl.volume_encode(to_dev(vol, dev), m, coder, ws)
    say("volume decode", H, Z, h, w, G, L, ws)
    dec, st = dl.volume_decode(bits, m, check=False)
    torch.cuda.synchronize()
    assert st == 0
    assert np.array_equal(dec.cpu().numpy(), vol)


def test_twelve_input_model_codes_slices_together(dev):
    layers = _layers(64, 7, k_in=12)
    m = dl.DeepModel(layers, dev)
    vol = _vol(5, 18, 22, 3)
    coder = dl.dlic_coder(2, 4)
    say("volume k12")
    bits = dl.volume_encode(to_dev(vol, dev), m, coder, 0)
    dec, st = dl.volume_decode(bits, m, check=False)
    torch.cuda.synchronize()
    assert st == 0 and np.array_equal(dec.cpu().numpy(), vol)
    # the body is every slice's image stream body, slice after slice
    parts = [dl.deep_encode(to_dev(vol[z], dev), m, coder).cpu().numpy().tobytes()
             for z in range(5)]
    counts = b"".join(p[oracle.HEADER_SIZE:oracle.HEADER_SIZE + 8] for p in parts)
    words = b"".join(p[oracle.HEADER_SIZE + 8:] for p in parts)
    assert bits.cpu().numpy().tobytes()[oracle.HEADER_SIZE:] == counts + words
    with pytest.raises(dl.DlicError):
        dl.volume_encode(to_dev(vol, dev), m, coder, 1)


def test_small_forced_grid_decodes_the_same(dev, net):
    H, layers, m = net
    vol = _vol(6, 30, 28, 21)
    bits = dl.volume_encode(to_dev(vol, dev), m, dl.dlic_coder(2, 4), 1)
    try:
        dl.dlic_set_deep_decode_grid(3)
        say("volume decode grid 3", H)
        dec, st = dl.volume_decode(bits, m, check=False)
        torch.cuda.synchronize()
        assert dl.dlic_deep_decode_grid() == 3
    finally:
        dl.dlic_set_deep_decode_grid(0)
    assert st == 0 and np.array_equal(dec.cpu().numpy(), vol)


def test_coded_length_near_ideal(dev, net):
    H, layers, m = net
    vol = _vol(4, 32, 40, 9)
    G, L = 1, 16
    bits = dl.volume_encode(to_dev(vol, dev), m, dl.dlic_coder(G, L), 1)
    torch.cuda.synchronize()
    logits = sm.deep_forward_bf16(vo.volume_features(vol, 1).reshape(-1, 21), layers)
    ideal = sm.ideal_bits_softmax(logits, vol.reshape(-1))
    payload = 8 * (bits.numel() - oracle.HEADER_SIZE - 4 * 4 * G)
    assert payload <= ideal + vol.size * (math.log2(65536 / 65280) + 0.02) + 4 * G * 32 * L


def test_errors(dev, net):
    H, layers, m = net
    vol = _vol(3, 14, 18, 4)
    coder = dl.dlic_coder(2, 4)
    bits = dl.volume_encode(to_dev(vol, dev), m, coder, 1)
    other = dl.DeepModel([(W, b + np.float32(0.01)) for W, b in layers], dev)
    say("volume wrong model")
    _, st = dl.volume_decode(bits, other, check=False)
    assert st == dl.DLIC_ERR_MODEL_MISMATCH
    say("volume truncated")
    _, st = dl.volume_decode(bits[:-2], m, check=False)
    assert st == dl.DLIC_ERR_CORRUPT
    # geometry the stream does not hold: another window shift or slice split
    out = torch.empty((3, 14, 18), dtype=torch.uint8, device=dev)
    stt = torch.zeros(1, dtype=torch.int32, device=dev)
    for z, h, ws in [(3, 14, 2), (6, 7, 1)]:
        wsb = dl.dlic_volume_workspace(m, z, h, 18, coder, 1)
        wsp = torch.empty(wsb, dtype=torch.uint8, device=dev)
        say("volume geometry", z, h, ws)
        rc = dl.lib().dlic_volume_decode(dl.ctypes.byref(m.c), dl.ctypes.byref(coder), bits.data_ptr(),
                                         bits.numel(), out.data_ptr(), z, h, 18, ws, stt.data_ptr(),
                                         wsp.data_ptr(), wsb, None)
        torch.cuda.synchronize()
        assert rc == 0 and int(stt.item()) == dl.DLIC_ERR_CORRUPT
    # arguments out of range are refused before any launch
    for z, ws in [(0, 1), (4096, 1), (3, 16), (3, -1)]:
        rc = dl.lib().dlic_volume_encode(dl.ctypes.byref(m.c), dl.ctypes.byref(coder), out.data_ptr(),
                                         z, 14, 18, ws, out.data_ptr(), 1 << 20, stt.data_ptr(),
                                         out.data_ptr(), 1 << 20, None)
        assert rc == dl.DLIC_ERR_ARG
    # the image decoder refuses the 21-input model; the volume reader an image stream
    with pytest.raises(dl.DlicError):
        dl.deep_decode(bits, m)
    img_bits = dl.deep_encode(to_dev(vol[0], dev), dl.DeepModel(_layers(H, 3, k_in=12), dev), coder)
    with pytest.raises(dl.DlicError):
        dl.volume_decode(img_bits, m)


def test_scan_full_size(dev):
    # the 256x256x35 scan of the paper's MRI timing table, the 128-wide network,
    # window shift 1: round trip, and sampled logits against the oracle voxel by voxel
    layers = _layers(128, 77)
    m = dl.DeepModel(layers, dev)
    vol = synth.mri_volume(2024)
    coder = dl.dlic_coder(8, 8)
    say("volume full encode")
    d_vol = to_dev(vol, dev)
    bits = dl.volume_encode(d_vol, m, coder, 1)
    say("volume full decode")
    dec, st = dl.volume_decode(bits, m, check=False)
    torch.cuda.synchronize()
    assert st == 0 and torch.equal(dec, d_vol)
    say("volume full density")
    lg, _, _ = dl.volume_density(d_vol, m, 1)
    rng = np.random.default_rng(5)
    idx = rng.integers(0, vol.size, 1500)
    idx[:3] = [0, 256 * 256, vol.size - 1]
    got = lg[torch.from_numpy(idx).to(dev)].cpu().numpy().astype(np.float64)
    del lg
    zz, rem = np.divmod(idx, 256 * 256)
    yy, xx = np.divmod(rem, 256)
    feats = np.stack([vo.voxel_features(vol, z, y, x, 1) for z, y, x in zip(zz, yy, xx)])
    ref = sm.deep_forward_bf16(feats, layers)
    err = np.abs(got - ref) / np.maximum(1.0, np.abs(ref))
    assert err.max() <= 2.0 ** -6 and (err.max(axis=1) <= 2.0 ** -8).mean() >= 0.99


def test_slice_stamps_follow_the_wavefront(dev, net):
    # with WS = 2 slice z + 1 trails slice z by five steps and its last pixel's window
    # reads slice z's last pixel, so the slices complete in order after the start
    H, layers, m = net
    Z = 5
    vol = _vol(Z, 20, 24, 8)
    bits = dl.volume_encode(to_dev(vol, dev), m, dl.dlic_coder(2, 4), 2)
    say("volume stamps", H)
    dec, st = dl.volume_decode(bits, m, check=False)
    torch.cuda.synchronize()
    assert st == 0 and np.array_equal(dec.cpu().numpy(), vol)
    s = dl.dlic_deep_slice_stamps(Z + 1).astype(np.int64)
    assert np.all(s[1:] > s[0]) and np.all(np.diff(s[1:]) >= 0), s
    with pytest.raises(dl.DlicError):
        dl.dlic_deep_slice_stamps(5000)
