"""Row strips spread over the image (several strips per group): GPU encoder and decoders
against the oracle, bit for bit.

A group codes strips g, G + g, ... one after another with its lanes' states carried
over (Section II-B, rANS: several coder instances and bitstreams; Preprocessor: the
wavefront order).  The encoder's streams equal the oracle's byte for byte, the
table-driven decoder reads oracle-written streams, the network decoder returns the
image, and at 2048x1536 the 64 x 4 layout with two strips per group round-trips.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2207_05152_amd as dl
import synth
from gpu_util import cf_pack, dev, say, to_dev  # noqa: F401

pytestmark = pytest.mark.gpu

# (h, w, G, L, S): strips of 2..40 rows, lane counts of every coder form
CASES = [(12, 9, 2, 2, 2), (40, 37, 2, 4, 2), (70, 20, 3, 4, 3), (64, 64, 1, 32, 2),
         (90, 33, 2, 7, 4), (48, 100, 4, 1, 2), (33, 5, 1, 4, 16), (128, 70, 2, 64, 2)]


def _inputs(h, w, seed):
    tabs = synth.random_tables(37, seed).astype(np.int64)
    rng = np.random.default_rng(seed)
    tidx = rng.integers(0, len(tabs), size=(h, w))
    sym = synth.random_symbols_from_tables(tabs, tidx, seed + 1).astype(np.int64)
    c = tabs[tidx, sym]
    f = tabs[tidx, sym + 1] - c
    return tabs, tidx, sym, c, f


def _oracle_raw(h, w, G, L, S, c, f):
    streams = []
    for grp in oracle.canonical_order(h, w, G, L, strips=S):
        streams.append(oracle.rans_encode([(c[y, x], f[y, x]) for (y, x, _) in grp],
                                          [ln for (_, _, ln) in grp], L))
    return oracle.assemble(oracle.pack_header(h, w, G, L, flags=oracle.image_flags(S)), streams)


def _encode_cf(dev, h, w, coder, c, f):
    cap = dl.dlic_encode_bound(h, w, coder)
    out = torch.zeros(cap, dtype=torch.uint8, device=dev)
    olen = torch.zeros(1, dtype=torch.int64, device=dev)
    wsb = dl.dlic_encode_workspace(h, w, coder)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    dl.dlic_rans_encode_cf(coder, h, w, to_dev(cf_pack(c, f), dev), out, cap, olen, ws, wsb)
    torch.cuda.synchronize()
    return out[: int(olen.item())].cpu().numpy().tobytes()


def _decode_tables(dev, h, w, coder, tabs, tidx, raw):
    bits = to_dev(np.frombuffer(raw, dtype=np.uint8), dev)
    sym = torch.zeros((h, w), dtype=torch.uint8, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    wsb = dl.dlic_decode_workspace(h, w, coder)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    d_tab = to_dev(tabs.astype(np.uint32).view(np.int32), dev)
    d_idx = to_dev(tidx.astype(np.uint32).view(np.int32).ravel(), dev)
    dl.dlic_rans_decode_tables(coder, h, w, d_tab, len(tabs), d_idx, bits, len(raw), sym, st, ws,
                               wsb)
    torch.cuda.synchronize()
    return sym.cpu().numpy(), int(st.item())


@pytest.mark.parametrize("h,w,G,L,S", CASES)
def test_encode_bytes_equal_oracle(dev, h, w, G, L, S):
    tabs, tidx, sym, c, f = _inputs(h, w, 3000 + h * 7 + w + S)
    say("strips rans_encode_cf", h, w, G, L, S)
    got = _encode_cf(dev, h, w, dl.dlic_coder(G, L, S), c, f)
    assert got == _oracle_raw(h, w, G, L, S, c, f)


@pytest.mark.parametrize("h,w,G,L,S", CASES)
def test_decode_oracle_stream_with_tables(dev, h, w, G, L, S):
    tabs, tidx, sym, c, f = _inputs(h, w, 4000 + h * 7 + w + S)
    raw = _oracle_raw(h, w, G, L, S, c, f)
    say("strips rans_decode_tables", h, w, G, L, S)
    got, st = _decode_tables(dev, h, w, dl.dlic_coder(G, L, S), tabs, tidx, raw)
    assert st == 0
    assert np.array_equal(got, sym.astype(np.uint8))


def test_peek_reports_strips():
    raw = oracle.pack_header(96, 50, 4, 4, flags=oracle.image_flags(3))
    hd = dl.dlic_peek_header(raw)
    c = hd["coder"]
    assert (c.groups, c.lanes_per_group, c.strips) == (4, 4, 3)


@pytest.mark.parametrize("h,w,width,G,L,S", [
    (12, 9, 32, 2, 2, 2), (60, 90, 64, 3, 4, 2), (64, 200, 64, 4, 4, 4), (96, 130, 128, 6, 4, 2),
    (80, 60, 64, 2, 32, 2), (70, 64, 32, 1, 64, 2), (40, 50, 32, 2, 1, 5)])
def test_network_stream_equals_oracle_and_round_trips(dev, h, w, width, G, L, S):
    img = synth.synth_image(h, w, 11 + h + w + S)
    wts = synth.xavier_mlp((12, width, width, 15), 3)
    m = dl.Model(wts, dev)
    coder = dl.dlic_coder(G, L, S)
    say("strips encode", h, w, width, G, L, S)
    bits = dl.encode(to_dev(img, dev), m, coder)
    raw = bits.cpu().numpy().tobytes()
    # the GPU's intervals, coded by the oracle in the strips' canonical order
    _, cf, _ = dl.density(to_dev(img, dev), m)
    cfn = cf.cpu().numpy().view(np.uint32).astype(np.int64).reshape(h, w)
    c, f = cfn & 0xFFFF, (cfn >> 16) + 1
    want = _oracle_raw(h, w, G, L, S, c, f)
    assert raw[36:] == want[36:]
    assert raw[:36] == oracle.pack_header(h, w, G, L, dtype=0, h1=width, h2=width,
                                          fp=oracle.weights_fingerprint(wts),
                                          flags=oracle.image_flags(S))
    say("strips decode", h, w, width, G, L, S)
    dec, st = dl.decode(bits, m, check=False)
    torch.cuda.synchronize()
    assert st == 0
    assert np.array_equal(dec.cpu().numpy(), img)


def test_small_image_decodes_like_the_oracle(dev):
    """The oracle's own encode (FP64 network, FP32 tables) of a small image with strips,
    decoded on the GPU: the stream is the oracle's, not the GPU encoder's."""
    img = synth.synth_image(16, 12, 5)
    wts = synth.xavier_mlp((12, 32, 32, 15), 3)
    raw = oracle.encode_image(img, wts, oracle.OracleCoder(2, 2, 2))
    m = dl.Model(wts, dev)
    say("strips decode of an oracle stream")
    dec, st = dl.decode(to_dev(np.frombuffer(raw, dtype=np.uint8), dev), m, check=False)
    torch.cuda.synchronize()
    assert st == 0 and np.array_equal(dec.cpu().numpy(), img)


def test_full_size_two_strips_round_trip(dev):
    """2048x1536, 12-64-64-15 FP32, 64 groups x 4 lanes (256 lanes), 2 strips per group:
    first and last group byte-identical to the oracle's coding of the GPU intervals, and
    the decode returns the image."""
    h, w, G, L, S = 1536, 2048, 64, 4, 2
    img = synth.synth_image(h, w, 1)
    wts = synth.xavier_mlp((12, 64, 64, 15), 3)
    m = dl.Model(wts, dev)
    d_img = to_dev(img, dev)
    coder = dl.dlic_coder(G, L, S)
    say("strips full size encode")
    bits = dl.encode(d_img, m, coder)
    raw = bits.cpu().numpy().tobytes()
    _, cf, _ = dl.density(d_img, m)
    cfn = cf.cpu().numpy().view(np.uint32).astype(np.int64).reshape(h, w)
    c, f = cfn & 0xFFFF, (cfn >> 16) + 1
    parts = oracle.split_streams(raw, G)
    order = oracle.canonical_order(h, w, G, L, only={0, G - 1}, strips=S)
    for g in (0, G - 1):
        grp = order[g]
        want = oracle.rans_encode([(c[y, x], f[y, x]) for (y, x, _) in grp],
                                  [ln for (_, _, ln) in grp], L)
        assert parts[g] == want, g
    say("strips full size decode")
    dec, st = dl.decode(bits, m, check=False)
    torch.cuda.synchronize()
    assert st == 0
    assert np.array_equal(dec.cpu().numpy(), img)


@pytest.fixture
def delays():
    yield dl.dlic_set_decode_delays
    dl.dlic_set_decode_delays(0, 0)


@pytest.mark.parametrize("h,w,width,G,L,S", [(96, 160, 64, 4, 4, 2), (120, 90, 64, 2, 32, 3)])
@pytest.mark.parametrize("seed,max_cycles", [(3, 3000), (4, 20000)])
def test_round_trip_under_injected_delays(dev, delays, h, w, width, G, L, S, seed, max_cycles):
    img = synth.synth_image(h, w, 23 + seed)
    m = dl.Model(synth.xavier_mlp((12, width, width, 15), 3), dev)
    bits = dl.encode(to_dev(img, dev), m, dl.dlic_coder(G, L, S))
    delays(seed, max_cycles)
    say("strips delays", h, w, width, G, L, S, seed, max_cycles)
    dec, st = dl.decode(bits, m, check=False)
    torch.cuda.synchronize()
    assert st == 0
    assert np.array_equal(dec.cpu().numpy(), img)


def test_errors(dev):
    h, w = 40, 30
    img = synth.synth_image(h, w, 9)
    m = dl.Model(synth.xavier_mlp((12, 32, 32, 15), 3), dev)
    bits = dl.encode(to_dev(img, dev), m, dl.dlic_coder(2, 4, 2))
    # a header whose strips disagree with the layout passed in: status 3, no wait
    raw = bytearray(bits.cpu().numpy().tobytes())
    raw[7] = 0x20
    say("strips wrong flags")
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    out = torch.empty((h, w), dtype=torch.uint8, device=dev)
    coder = dl.dlic_coder(2, 4, 2)
    wsb = dl.dlic_decode_workspace(h, w, coder)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    dl.dlic_decode(m.c, coder, to_dev(np.frombuffer(bytes(raw), np.uint8), dev), len(raw), out, h,
                   w, st, ws, wsb)
    torch.cuda.synchronize()
    assert int(st.item()) == 3
    # a damaged payload: reported, and every wait ends
    raw = bytearray(bits.cpu().numpy().tobytes())
    raw[60] ^= 0xFF
    raw[-3] ^= 0x5A
    say("strips damaged payload")
    dec, st2 = dl.decode(to_dev(np.frombuffer(bytes(raw), np.uint8), dev), m, check=False)
    torch.cuda.synchronize()
    assert st2 != 0 or not np.array_equal(dec.cpu().numpy(), img)


@pytest.mark.parametrize("dtype", ["fp32", "bf16", "fp8", "fp8a8"])
@pytest.mark.parametrize("width,S", [(64, 2), (128, 2), (64, 3), (128, 5)])
def test_every_precision_round_trips_with_strips(dev, dtype, width, S):
    """Each network form of the decoder (4-pixel FP32, BF16, FP8 weights, FP8 weights and
    activations) in its two-strip and its any-number-of-strips kernel."""
    h, w, G, L = 120, 150, 4, 4
    img = synth.synth_image(h, w, 31 + width + S)
    wts = synth.xavier_mlp((12, width, width, 15), 3)
    cal = [to_dev(synth.synth_image(64, 64, 1000 + i), dev) for i in range(2)]
    m = dl.Model(wts, dev, dtype=dtype, calibration=cal if dtype == "fp8a8" else None)
    coder = dl.dlic_coder(G, L, S)
    say("strips precision", dtype, width, S)
    bits = dl.encode(to_dev(img, dev), m, coder)
    dec, st = dl.decode(bits, m, check=False)
    torch.cuda.synchronize()
    assert st == 0
    assert np.array_equal(dec.cpu().numpy(), img)
