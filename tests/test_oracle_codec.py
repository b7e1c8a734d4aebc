"""Pins of the oracle's whole-image codec and container (CPU)."""
import math

import numpy as np
import pytest

import oracle
import synth


def test_fnv1a_vectors(golden):
    for ln in golden("fnv1a64.txt"):
        text, want = ln.rsplit(":", 1)
        data = np.frombuffer(text.strip().strip('"').encode("ascii"), dtype=np.uint8)
        assert oracle.fingerprint([data]) == int(want.strip(), 16)


def test_header_round_trip():
    hdr = oracle.pack_header(1536, 2048, 8, 32, dtype=1, h1=64, h2=64, fp=0x0123456789ABCDEF)
    assert len(hdr) == oracle.HEADER_SIZE == 36
    p = oracle.parse_header(hdr)
    assert (p["h"], p["w"], p["groups"], p["lanes"], p["dtype"], p["h1"], p["h2"]) == \
        (1536, 2048, 8, 32, 1, 64, 64)
    assert p["fingerprint"] == 0x0123456789ABCDEF and p["skew"] == 3 and p["prob_bits"] == 16


def _header_cases(golden):
    cases, container = [], None
    for ln in golden("header_v1.txt"):
        left, right = ln.split(":")
        raw = bytes.fromhex(right.replace(" ", ""))
        f = left.split()
        if f[0] == "container":
            container = ([int(v, 16) for v in f[1:]], raw)
        else:
            h, w, g, l, dt, h1, h2 = (int(v) for v in f[:7])
            cases.append(((h, w, g, l, dt, h1, h2, int(f[7], 16)), raw))
    return cases, container


def test_header_bytes_match_hand_written_golden(golden):
    cases, (words, tail) = _header_cases(golden)
    assert len(cases) == 3
    for (h, w, g, l, dt, h1, h2, fp), raw in cases:
        assert oracle.pack_header(h, w, g, l, dtype=dt, h1=h1, h2=h2, fp=fp) == raw
        p = oracle.parse_header(raw)
        assert (p["h"], p["w"], p["groups"], p["lanes"], p["dtype"], p["h1"], p["h2"],
                p["fingerprint"]) == (h, w, g, l, dt, h1, h2, fp)
    hdr = cases[1][1]
    full = oracle.assemble(hdr, [words])
    assert full == hdr + tail
    assert oracle.split_streams(full, 1) == [words]


def test_c0_round_trip_and_rate(c0_inputs):
    img, w = c0_inputs
    bits = oracle.encode_image(img, w, oracle.OracleCoder(1, 32))
    assert np.array_equal(oracle.decode_image(bits, w), img)
    n = img.size
    payload = 8 * (len(bits) - oracle.HEADER_SIZE - 4)
    ideal = oracle.ideal_bits_image(img, w)
    c, f = oracle.cf_for_image(img, w)
    cost = math.fsum((-np.log2(f / 65536.0)).tolist())
    # table rule loses at most log2(M/M') per pixel (+ the FP32 CDF's tiny error)
    assert cost <= ideal + n * math.log2(65536 / 65280) + 1e-3 * n
    assert cost - 1.0 <= payload <= cost + 32 * 32 + 0.02 * n


@pytest.mark.parametrize("h,w,g,lanes", [(1, 1, 1, 32), (1, 5, 1, 32), (5, 1, 1, 32),
                                          (2, 3, 2, 32), (5, 7, 1, 4), (33, 4, 2, 32),
                                          (40, 9, 3, 4), (3, 5, 4, 2)])
def test_odd_shapes_round_trip(h, w, g, lanes):
    img = synth.synth_image(h, w, 7 + h * w)
    wts = synth.xavier_mlp((12, 8, 8, 15), 11)
    bits = oracle.encode_image(img, wts, oracle.OracleCoder(g, lanes))
    assert np.array_equal(oracle.decode_image(bits, wts), img)


def test_wrong_model_is_refused(c0_inputs):
    img, w = c0_inputs
    img = img[:8, :8]
    bits = oracle.encode_image(img, w, oracle.OracleCoder(1, 32))
    other = dict(w); other["b3"] = w["b3"] + np.float32(1e-3)
    with pytest.raises(ValueError):
        oracle.decode_image(bits, other)
