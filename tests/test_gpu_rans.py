"""rANS parity: GPU coder vs the oracle on identical seeded tables (bit-exact)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2207_05152_amd as dl
import synth
from gpu_util import cf_pack, dev, say, to_dev  # noqa: F401

pytestmark = pytest.mark.gpu

CASES = [(64, 64, 1, 32), (70, 37, 2, 32), (300, 129, 3, 7), (1, 1, 1, 32), (2, 3, 1, 32),
         (9, 200, 2, 64), (40, 5, 4, 1), (512, 3, 2, 32)]


def _inputs(h, w, seed):
    tabs = synth.random_tables(37, seed).astype(np.int64)
    rng = np.random.default_rng(seed)
    tidx = rng.integers(0, len(tabs), size=(h, w))
    sym = synth.random_symbols_from_tables(tabs, tidx, seed + 1).astype(np.int64)
    c = tabs[tidx, sym]
    f = tabs[tidx, sym + 1] - c
    return tabs, tidx, sym, c, f


def _oracle_stream(h, w, G, L, c, f, groups=None):
    streams = []
    for g, grp in enumerate(oracle.canonical_order(h, w, G, L, only=groups)):
        if groups is not None and g not in groups:
            streams.append(None)
            continue
        streams.append(oracle.rans_encode([(c[y, x], f[y, x]) for (y, x, _) in grp],
                                          [ln for (_, _, ln) in grp], L))
    return streams


def _gpu_encode_cf(dev, h, w, coder, c, f):
    cap = dl.dlic_encode_bound(h, w, coder)
    out = torch.zeros(cap, dtype=torch.uint8, device=dev)
    olen = torch.zeros(1, dtype=torch.int64, device=dev)
    wsb = dl.dlic_encode_workspace(h, w, coder)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    d_cf = to_dev(cf_pack(c, f), dev)
    dl.dlic_rans_encode_cf(coder, h, w, d_cf, out, cap, olen, ws, wsb)
    torch.cuda.synchronize()
    return out[: int(olen.item())].cpu().numpy().tobytes()


def _gpu_decode_tables(dev, h, w, coder, tabs, tidx, raw):
    bits = to_dev(np.frombuffer(raw, dtype=np.uint8), dev)
    sym = torch.zeros((h, w), dtype=torch.uint8, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    wsb = dl.dlic_decode_workspace(h, w, coder)
    ws = torch.empty(wsb, dtype=torch.uint8, device=dev)
    d_tab = to_dev(tabs.astype(np.uint32).view(np.int32), dev)
    d_idx = to_dev(tidx.astype(np.uint32).view(np.int32).ravel(), dev)
    dl.dlic_rans_decode_tables(coder, h, w, d_tab, len(tabs), d_idx, bits, len(raw), sym, st, ws, wsb)
    torch.cuda.synchronize()
    return sym.cpu().numpy(), int(st.item())


@pytest.mark.parametrize("h,w,G,L", CASES)
def test_encode_bytes_equal_oracle(dev, h, w, G, L):
    tabs, tidx, sym, c, f = _inputs(h, w, 1000 + h * 7 + w)
    want = oracle.assemble(oracle.pack_header(h, w, G, L), _oracle_stream(h, w, G, L, c, f))
    say("rans_encode_cf", h, w, G, L)
    got = _gpu_encode_cf(dev, h, w, dl.dlic_coder(G, L), c, f)
    assert got == want


@pytest.mark.parametrize("h,w,G,L", CASES)
def test_decode_oracle_stream_with_tables(dev, h, w, G, L):
    tabs, tidx, sym, c, f = _inputs(h, w, 2000 + h * 7 + w)
    raw = oracle.assemble(oracle.pack_header(h, w, G, L), _oracle_stream(h, w, G, L, c, f))
    say("rans_decode_tables", h, w, G, L)
    got, st = _gpu_decode_tables(dev, h, w, dl.dlic_coder(G, L), tabs, tidx, raw)
    assert st == 0
    assert np.array_equal(got, sym.astype(np.uint8))


@pytest.mark.parametrize("G,L", [(8, 32), (64, 4)])
def test_full_size_layout_sampled_groups(dev, G, L):
    # The 2048x1536 image in 256-lane layouts: GPU stream of the first and the
    # last group byte-identical to the oracle's; every group decodes back.
    h, w = 1536, 2048
    tabs, tidx, sym, c, f = _inputs(h, w, 77)
    say("rans_encode_cf full size", h, w, G, L)
    got = _gpu_encode_cf(dev, h, w, dl.dlic_coder(G, L), c, f)
    parts = oracle.split_streams(got, G)
    want = _oracle_stream(h, w, G, L, c, f, groups={0, G - 1})
    assert parts[0] == want[0] and parts[G - 1] == want[G - 1]
    say("rans_decode_tables full size", h, w, G, L)
    dec, st = _gpu_decode_tables(dev, h, w, dl.dlic_coder(G, L), tabs, tidx, got)
    assert st == 0 and np.array_equal(dec, sym.astype(np.uint8))


def test_corrupt_and_truncated_streams_are_reported(dev):
    h, w, G, L = 64, 64, 2, 32
    tabs, tidx, sym, c, f = _inputs(h, w, 5)
    raw = oracle.assemble(oracle.pack_header(h, w, G, L), _oracle_stream(h, w, G, L, c, f))
    coder = dl.dlic_coder(G, L)
    bad = bytearray(raw)
    bad[len(raw) // 2] ^= 0x5A
    say("corrupt payload")
    dec, st = _gpu_decode_tables(dev, h, w, coder, tabs, tidx, bytes(bad))
    assert st == dl.DLIC_ERR_CORRUPT or not np.array_equal(dec, sym.astype(np.uint8))
    say("truncated")
    _, st = _gpu_decode_tables(dev, h, w, coder, tabs, tidx, raw[:-2])
    assert st == dl.DLIC_ERR_CORRUPT
    say("bad magic")
    _, st = _gpu_decode_tables(dev, h, w, coder, tabs, tidx, b"X" + raw[1:])
    assert st == dl.DLIC_ERR_CORRUPT
