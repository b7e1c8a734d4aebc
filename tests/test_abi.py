"""The C-ABI library loads and exports what include/dlic.h declares; host-only
helpers agree with the oracle (CPU, no device calls)."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import paper_2207_05152_amd as dl
from conftest import ROOT


def _declared():
    src = open(os.path.join(ROOT, "include", "dlic.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dlic_\w+)\s*\(", src)))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(dl.LIB_PATH)
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(dl.EXPORTS)


def test_noalloc_limit_macro_matches_binding():
    src = open(os.path.join(ROOT, "include", "dlic.h")).read()
    m = re.search(r"#define DLIC_DECODE_NOALLOC_BYTES \(\(size_t\)(\d+) << (\d+)\)", src)
    assert m, "DLIC_DECODE_NOALLOC_BYTES not found"
    assert int(m.group(1)) << int(m.group(2)) == dl.DECODE_NOALLOC_BYTES == 8 << 20


def test_constant_tables_match_oracle_bit_for_bit():
    S, D, beta, scale = dl.dlic_host_constants()
    So, Do = oracle.sigma_lut32()
    assert np.array_equal(S.view(np.uint32), So.view(np.uint32))
    assert np.array_equal(D.view(np.uint32), Do.view(np.uint32))
    assert np.array_equal(beta.view(np.uint32), oracle.beta32().view(np.uint32))
    assert np.array_equal(scale.view(np.uint32), oracle.scale32().view(np.uint32))


def test_fnv_and_fingerprint_match_oracle(golden):
    for ln in golden("fnv1a64.txt"):
        text, want = ln.rsplit(":", 1)
        assert dl.dlic_fnv1a64(dl.FNV_OFFSET, text.strip().strip('"').encode()) == int(want, 16)
    import synth
    w = synth.xavier_mlp((12, 32, 32, 15), 7)
    h = dl.FNV_OFFSET
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        h = dl.dlic_fnv1a64(h, w[k].tobytes())
    assert h == oracle.weights_fingerprint(w)


def test_bounds_and_workspace():
    c = dl.dlic_coder(8, 32)
    assert dl.dlic_encode_bound(1536, 2048, c) == 36 + 4 * 8 + 2 * (1536 * 2048 + 2 * 32 * 8)
    assert dl.dlic_encode_workspace(1536, 2048, c) >= 6 * 1536 * 2048
    assert dl.dlic_decode_workspace(1536, 2048, c) >= 4 * 8 * (2048 + 3 * 1536 - 3)
    assert dl.dlic_encode_bound(10, 10, dl.dlic_coder(6, 32)) == 0      # H < 2G
    assert dl.dlic_encode_bound(10, 10, dl.dlic_coder(1, 65)) == 0      # L > 64
    assert dl.dlic_encode_bound(257, 10, dl.dlic_coder(1, 32)) == 0     # > 256 rows per group


def test_volume_bound_workspace_and_peek():
    # the stacked image's bound: z h rows, z G groups
    c = dl.dlic_coder(8, 8)
    L = dl.lib()
    assert L.dlic_volume_encode_bound(35, 256, 256, ctypes.byref(c)) == \
        36 + 4 * 8 * 35 + 2 * (35 * 256 * 256 + 2 * 8 * 8 * 35)
    assert L.dlic_volume_encode_bound(0, 256, 256, ctypes.byref(c)) == 0
    assert L.dlic_volume_encode_bound(4096, 256, 256, ctypes.byref(c)) == 0
    assert L.dlic_volume_encode_bound(200, 256, 256, ctypes.byref(c)) == 0   # 1600 groups
    ptrs = (ctypes.c_void_p * 6)(*([16] * 6))       # never dereferenced by these host calls
    m = dl.dlic_deep_model(128, 21, ptrs, ptrs, 0, 8)
    assert L.dlic_volume_workspace(ctypes.byref(m), 35, 256, 256, ctypes.byref(c), 1) >= 35 * 256 * 512
    m12 = dl.dlic_deep_model(128, 21, ptrs, ptrs, 0, 12)
    # 12-bit decoding keeps each row's table and logits: 24 KB per row
    assert L.dlic_volume_workspace(ctypes.byref(m12), 35, 256, 256, ctypes.byref(c), 1) >= \
        35 * 256 * (8192 + 16384)
    for bad in (dl.dlic_deep_model(96, 21, ptrs, ptrs, 0, 8), dl.dlic_deep_model(128, 21, ptrs, ptrs, 0, 10),
                dl.dlic_deep_model(128, 13, ptrs, ptrs, 0, 8)):
        assert L.dlic_volume_workspace(ctypes.byref(bad), 35, 256, 256, ctypes.byref(c), 1) == 0
    hdr = oracle.pack_header(35 * 256, 256, 35 * 8, 8, dtype=1, h1=128, h2=128, n_mix=0, k_in=21,
                             flags=oracle.volume.volume_flags(35, 2))
    p = dl.dlic_peek_volume(hdr)
    assert (p["z"], p["h"], p["ws"], p["k_in"], p["coder"].groups, p["coder"].lanes_per_group) == \
        (35, 256, 2, 21, 8, 8)
    with pytest.raises(dl.DlicError):   # an image's header holds no slice count
        dl.dlic_peek_volume(oracle.pack_header(256, 256, 8, 8))
    with pytest.raises(dl.DlicError):   # rows not a multiple of the slices
        dl.dlic_peek_volume(oracle.pack_header(257, 256, 35, 8, flags=35))


@pytest.mark.parametrize("depth", [8, 12])
def test_host_scale_matches_oracle_bit_for_bit(depth):
    got = dl.dlic_host_scale(depth)
    want = oracle.scale(np.arange(1 << depth), depth).astype(np.float32)
    assert got.shape == want.shape and np.array_equal(got.view(np.uint32), want.view(np.uint32))
    with pytest.raises(dl.DlicError):
        dl.dlic_host_scale(10)


def test_peek_header_reads_oracle_header():
    hdr = oracle.pack_header(1536, 2048, 8, 32, dtype=0, h1=64, h2=64, fp=0xFEEDFACE01234567)
    raw = hdr + bytes(4 * 8)
    p = dl.dlic_peek_header(raw)
    assert (p["h"], p["w"], p["coder"].groups, p["coder"].lanes_per_group, p["h1"], p["h2"]) == \
        (1536, 2048, 8, 32, 64, 64)
    assert p["fingerprint"] == 0xFEEDFACE01234567
    with pytest.raises(dl.DlicError):
        dl.dlic_peek_header(b"XLIC" + raw[4:])
    with pytest.raises(dl.DlicError):
        dl.dlic_peek_header(raw[:20])


def test_peek_header_reads_golden_bytes(golden):
    for ln in golden("header_v1.txt"):
        left, right = ln.split(":")
        f = left.split()
        if f[0] == "container":
            continue
        h, w, g, l, dt, h1, h2 = (int(v) for v in f[:7])
        p = dl.dlic_peek_header(bytes.fromhex(right.replace(" ", "")))
        assert (p["h"], p["w"], p["coder"].groups, p["coder"].lanes_per_group, p["dtype"],
                p["h1"], p["h2"], p["fingerprint"]) == (h, w, g, l, dt, h1, h2, int(f[7], 16))


def _quant_inputs():
    import synth
    from oracle import lowp
    w = synth.xavier_mlp((12, 128, 128, 15), 3)
    rng = np.random.default_rng(11)
    codes = np.arange(0x7F)
    vals = lowp.e4m3_value(codes)
    mids = (vals[1:] + vals[:-1]) / 2
    # a matrix whose scale is exactly 1: e4m3 ties, subnormals, zeros, saturation
    edge = np.concatenate([[448.0], vals, -vals, mids, -mids, [0.0, -0.0, 2 ** -10, 3 * 2 ** -10]])
    bf_ties = (np.arange(300, dtype=np.uint32) << 16 | 0x8000).view(np.float32)
    return [w["W1"], w["W2"], w["W3"], rng.standard_normal((7, 9)).astype(np.float32) * 1e-3,
            edge.astype(np.float32), bf_ties]


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_quantize_weights_matches_oracle(dtype):
    from oracle import lowp
    code = dl.DTYPES[dtype]
    for w in _quant_inputs():
        got, s = dl.dlic_quantize_weights(code, w)
        want, ws = lowp.quantize_matrix(w, dtype)
        assert got.dtype == want.dtype
        np.testing.assert_array_equal(got, want)
        assert np.float32(s).view(np.uint32) == np.float32(ws).view(np.uint32)


def test_quantize_weights_rejects_bad_input():
    lib = dl.lib()
    w = np.ones(4, np.float32)
    out = np.empty(4, np.uint16)
    sc = np.zeros(1, np.float32)
    assert lib.dlic_quantize_weights(dl.DLIC_FP32, w.ctypes.data, 4, out.ctypes.data,
                                     sc.ctypes.data) == dl.DLIC_ERR_ARG
    assert lib.dlic_quantize_weights(dl.DLIC_BF16, w.ctypes.data, 0, out.ctypes.data,
                                     sc.ctypes.data) == dl.DLIC_ERR_ARG
    w[2] = np.inf
    assert lib.dlic_quantize_weights(dl.DLIC_BF16, w.ctypes.data, 4, out.ctypes.data,
                                     sc.ctypes.data) == dl.DLIC_ERR_ARG
    assert lib.dlic_quantize_weights(dl.DLIC_FP8_E4M3, np.ones(4, np.float32).ctypes.data, 4,
                                     out.ctypes.data, None) == dl.DLIC_ERR_ARG


def test_device_entry_points_reject_bad_arguments_before_any_device_work():
    # every check below happens on the host, before the library touches a
    # device pointer (the dummies are never dereferenced)
    lib = dl.lib()
    P = 64  # a non-null dummy address
    m = dl.dlic_model(12, 32, 32, 15, dl.DLIC_FP32, 0, P, P, P, P, P, P, None, 0)
    c = dl.dlic_coder(1, 32)
    ctypes_ = ctypes
    enc = lambda h, w, mm, cc, cap=1 << 30, ws=1 << 30: lib.dlic_encode(
        ctypes_.byref(mm), ctypes_.byref(cc), P, h, w, P, cap, P, P, ws, None)
    dec = lambda h, w, mm, cc, n=1 << 20, ws=1 << 30: lib.dlic_decode(
        ctypes_.byref(mm), ctypes_.byref(cc), P, n, P, h, w, P, P, ws, None)
    assert enc(0, 5, m, c) == dl.DLIC_ERR_ARG            # empty image
    assert enc(5, 0, m, c) == dl.DLIC_ERR_ARG
    assert dec(0, 5, m, c) == dl.DLIC_ERR_ARG
    assert enc(8, 8, m, dl.dlic_coder(1, 65)) == dl.DLIC_ERR_UNSUPPORTED   # lanes
    assert enc(8, 8, m, dl.dlic_coder(5, 32)) == dl.DLIC_ERR_UNSUPPORTED   # rows per group < 2
    assert enc(600, 8, m, dl.dlic_coder(2, 32)) == dl.DLIC_ERR_UNSUPPORTED  # 300 rows per group
    assert enc(8, 8, m, c, cap=10) == dl.DLIC_ERR_CAPACITY
    assert enc(8, 8, m, c, ws=10) == dl.DLIC_ERR_CAPACITY
    assert dec(8, 8, m, c, ws=4) == dl.DLIC_ERR_CAPACITY
    bad = dl.dlic_model(12, 48, 48, 15, dl.DLIC_FP32, 0, P, P, P, P, P, P, None, 0)
    assert enc(8, 8, bad, c) == dl.DLIC_ERR_UNSUPPORTED  # width 48
    bad = dl.dlic_model(12, 32, 32, 15, dl.DLIC_FP8_E4M3, 0, P, P, P, P, P, P, None, 0)
    assert enc(8, 8, bad, c) == dl.DLIC_ERR_ARG          # FP8 without scales
    bad = dl.dlic_model(12, 32, 32, 15, 9, 0, P, P, P, P, P, P, None, 0)
    assert enc(8, 8, bad, c) == dl.DLIC_ERR_UNSUPPORTED  # unknown dtype
    bad = dl.dlic_model(11, 32, 32, 15, dl.DLIC_FP32, 0, P, P, P, P, P, P, None, 0)
    assert enc(8, 8, bad, c) == dl.DLIC_ERR_ARG          # window size


def test_w8a8_multipliers_match_oracle():
    from oracle import lowp
    rng = np.random.default_rng(12)
    vals = np.concatenate([[1.0, 448.0, 449.0, 224.0, 0.0, -1.0, 1e-6, 3.5e4],
                           np.exp(rng.uniform(-12, 8, 300))]).astype(np.float32)
    for i in range(0, len(vals) - 2, 3):
        got = dl.dlic_w8a8_multipliers(vals[i:i + 3])
        want = [lowp.w8a8_multiplier(float(v)) for v in vals[i:i + 3]]
        np.testing.assert_array_equal(got, np.array(want, np.float32))


def test_strip_layouts_host_checks():
    """Strips per group: limits, workspace of one record row per strip, header peek."""
    one = dl.dlic_coder(4, 4)
    two = dl.dlic_coder(4, 4, 2)
    assert dl.dlic_encode_bound(64, 10, two) == dl.dlic_encode_bound(64, 10, one) > 0
    assert dl.dlic_decode_workspace(64, 10, two) >= 2 * dl.dlic_decode_workspace(64, 10, one) - 256
    assert dl.dlic_encode_bound(15, 10, dl.dlic_coder(4, 4, 2)) == 0     # strips of < 2 rows
    assert dl.dlic_encode_bound(64, 10, dl.dlic_coder(1, 4, 17)) == 0    # > 16 strips
    assert dl.dlic_encode_bound(64, 10, dl.dlic_coder(1, 4, -1)) == 0
    assert dl.dlic_encode_bound(600, 10, dl.dlic_coder(1, 4, 2)) == 0    # 300-row strips
    assert dl.dlic_encode_bound(600, 10, dl.dlic_coder(1, 4, 3)) > 0     # 200-row strips
    # the deep network's codecs code one strip per group (the workspace call reads
    # only the model's sizes and that its pointers are set)
    class _M:
        c = dl.dlic_deep_model(hidden=64, k_in=12, depth=8)
    for i in range(dl.DEEP_LAYERS):
        _M.c.d_w[i] = 256 * (i + 1)
        _M.c.d_b[i] = 256 * (i + 9)
    assert dl.dlic_deep_workspace(_M, 64, 10, one, 0) > 0
    assert dl.dlic_deep_workspace(_M, 64, 10, two, 0) == 0
