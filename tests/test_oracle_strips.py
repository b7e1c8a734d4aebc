"""Pins of the row-strip layout (several strips per group) in the oracle (CPU).

A group may code S row strips spread over the image, its lanes' states carrying
from one strip to the next (Section II-B, rANS: several coder instances, each
with its own bitstream; Preprocessor: the wavefront order).  The layout is a
reading of ours; it is pinned by a hand-derived order, by invariants that hold
at any size, by hand-written header bytes and by round trips whose decoder
visits the strips in dependency order.
"""
import numpy as np
import pytest

import oracle
import synth


def _golden_order(golden):
    out = []
    for ln in golden("strips_order.txt"):
        left, right = ln.split(":")
        out.append([tuple(int(v) for v in t.split(",")) for t in right.split()])
    return out


def test_order_matches_hand_derived_golden(golden):
    assert oracle.group_rows(6, 4) == [0, 1, 3, 4, 6]
    assert oracle.group_strips(2, 2, 0) == [0, 2] and oracle.group_strips(2, 2, 1) == [1, 3]
    assert oracle.canonical_order(6, 4, 2, 2, strips=2) == _golden_order(golden)


@pytest.mark.parametrize("h,w,g,lanes,s", [(6, 4, 2, 2, 2), (48, 5, 4, 4, 2), (70, 9, 2, 32, 3),
                                            (13, 7, 3, 2, 4), (8, 3, 1, 4, 2), (16, 2, 2, 1, 8)])
def test_order_invariants(h, w, g, lanes, s):
    order = oracle.canonical_order(h, w, g, lanes, strips=s)
    rows = oracle.group_rows(h, g * s)
    seen = set()
    for gi, grp in enumerate(order):
        pos = 0
        for b in oracle.group_strips(g, s, gi):
            n = (rows[b + 1] - rows[b]) * w
            seg = grp[pos:pos + n]
            keys = []
            for (y, x, lane) in seg:
                assert rows[b] <= y < rows[b + 1]
                assert lane == (y - rows[b]) % lanes
                keys.append((x + 3 * y, (y - rows[b]) // lanes, lane))
                seen.add((y, x))
            assert keys == sorted(keys) and len(set(keys)) == n
            pos += n
        assert pos == len(grp)
    assert len(seen) == h * w


def test_one_strip_is_the_contiguous_layout():
    assert oracle.canonical_order(70, 9, 2, 4, strips=1) == oracle.canonical_order(70, 9, 2, 4)


def test_image_flags_and_header_bytes():
    assert oracle.image_flags(1) == 0 and oracle.image_flags(2) == 0x1000
    assert oracle.image_flags(16) == 0xF000
    assert oracle.image_strips(0) == 1 and oracle.image_strips(0x1000) == 2
    with pytest.raises(ValueError):
        oracle.image_strips(0x0023)      # a volume's flags (Z = 35)
    with pytest.raises(ValueError):
        oracle.image_flags(17)
    # bytes 6..7 hold the flags, little-endian: S = 2 gives 00 10
    hdr = oracle.pack_header(1536, 2048, 64, 4, dtype=0, h1=64, h2=64, fp=0x0123456789ABCDEF,
                             flags=oracle.image_flags(2))
    want = bytes.fromhex("444c4943 0100 0010 00060000 00080000 0c 05 00 03 4000 4000 10 04 4000 "
                         "efcdab8967452301".replace(" ", ""))
    assert hdr == want


@pytest.mark.parametrize("h,w,g,lanes,s", [(6, 4, 2, 2, 2), (12, 9, 2, 2, 2), (9, 5, 1, 4, 3),
                                            (16, 6, 2, 1, 4), (20, 3, 3, 2, 2)])
def test_round_trip_with_strips(h, w, g, lanes, s):
    img = synth.synth_image(h, w, 5 + h * w + s)
    wts = synth.xavier_mlp((12, 8, 8, 15), 11)
    coder = oracle.OracleCoder(g, lanes, s)
    bits = oracle.encode_image(img, wts, coder)
    assert oracle.parse_header(bits)["flags"] == oracle.image_flags(s)
    assert np.array_equal(oracle.decode_image(bits, wts), img)


def test_strips_change_the_stream_but_not_its_symbols():
    """The same (c, f) sequence per group, reordered: S = 2 and S = 1 streams differ,
    while each group's symbol multiset is that of its rows."""
    img = synth.synth_image(12, 9, 77)
    wts = synth.xavier_mlp((12, 8, 8, 15), 11)
    a = oracle.encode_image(img, wts, oracle.OracleCoder(2, 2, 1))
    b = oracle.encode_image(img, wts, oracle.OracleCoder(2, 2, 2))
    assert a[oracle.HEADER_SIZE:] != b[oracle.HEADER_SIZE:]
    assert np.array_equal(oracle.decode_image(a, wts), oracle.decode_image(b, wts))


def test_corrupt_strips_stream_is_refused():
    img = synth.synth_image(12, 9, 78)
    wts = synth.xavier_mlp((12, 8, 8, 15), 11)
    bits = bytearray(oracle.encode_image(img, wts, oracle.OracleCoder(2, 2, 2)))
    # claim one strip per group: the decoder then walks the symbols in another order,
    # and the lanes do not end at their initial state
    bits[7] = 0
    with pytest.raises(ValueError):
        oracle.decode_image(bytes(bits), wts)
