"""Pins of the oracle's 3-D window and 3-D wavefront (CPU): the vectorised window
against a voxel-by-voxel definition, the 2-D window as its special case, the lag
against its closed form and by brute force over every voxel (each lower-window
voxel is coded in an earlier step, one step less breaks it), the volume stream as
the concatenation of per-slice 2-D streams when the lower window carries no
weight, and round trips."""
import numpy as np
import pytest

import oracle
import synth
from oracle import softmax as sm
from oracle import volume as vo


def _layers(H=32, seed=5, bias=0.05, k_in=21):
    layers = synth.xavier_deep(H, seed, k_in=k_in)
    rng = np.random.default_rng(seed + 1)
    return [(W, rng.normal(0, bias, b.shape).astype(np.float32)) for W, b in layers]


def _vol(Z, H, W, seed):
    return np.random.default_rng(seed).integers(0, 256, (Z, H, W)).astype(np.uint8)


@pytest.mark.parametrize("ws", [0, 1, 2, 3])
def test_features_match_the_voxel_definition(ws):
    vol = _vol(3, 7, 6, 10 + ws)
    f = vo.volume_features(vol, ws)
    for z in range(3):
        for y in range(7):
            for x in range(6):
                assert np.array_equal(f[z, y, x], vo.voxel_features(vol, z, y, x, ws))


def test_lower_window_by_hand():
    # voxel (1, 4, 2), WS = 1: rows 2..4 of slice 0, columns 1..3, row by row
    vol = _vol(2, 6, 5, 3)
    f = vo.voxel_features(vol, 1, 4, 2, 1)
    want = [oracle.scale(int(vol[0, yy, xx])) for yy in (2, 3, 4) for xx in (1, 2, 3)]
    assert np.array_equal(f[12:], want)
    # outside the slice: 0; the first slice has no lower window
    g = vo.voxel_features(vol, 1, 0, 0, 1)
    # rows -2, -1 and column -1 fall outside; row 0 columns 0, 1 are the last two
    assert np.all(g[12:19] == 0)
    assert g[19] == oracle.scale(int(vol[0, 0, 0])) and g[20] == oracle.scale(int(vol[0, 0, 1]))
    assert np.all(vo.voxel_features(vol, 0, 3, 3, 1)[12:] == 0)


def test_same_slice_part_is_the_2d_window():
    vol = _vol(4, 9, 11, 7)
    f = vo.volume_features(vol, 2)
    for z in range(4):
        assert np.array_equal(f[z].reshape(-1, 21)[:, :12], oracle.causal_features(vol[z]))
    assert np.all(f[0, ..., 12:] == 0)


@pytest.mark.parametrize("ws", [0, 1, 2, 3, 4])
def test_lag_closed_form(ws):
    # largest lower offset dx + 3 dy is 1 + 3 (WS - 1); one more, never negative
    assert vo.lag(ws) == max(0, 3 * ws - 1)


@pytest.mark.parametrize("ws", [0, 1, 2, 3])
def test_wavefront_is_causal_and_tight(ws):
    Z, H, W = 3, 8, 7
    lg = vo.lag(ws)

    def step(z, y, x, lag):
        return x + oracle.SKEW * y + lag * z

    def violations(lag):
        bad = 0
        for z in range(1, Z):
            for y in range(H):
                for x in range(W):
                    for dy, dx in vo.lower_offsets(ws):
                        yy, xx = y + dy, x + dx
                        if 0 <= yy < H and 0 <= xx < W and step(z - 1, yy, xx, lag) >= step(z, y, x, lag):
                            bad += 1
        return bad

    assert violations(lg) == 0
    if lg > 0:
        assert violations(lg - 1) > 0
    # the same-slice window stays causal under any lag
    for dy, dx in oracle.NEIGHBOURS:
        assert dx + oracle.SKEW * dy < 0
    assert vo.n_steps_3d(Z, H, W, ws) == step(Z - 1, H - 1, W - 1, lg) + 1


def test_zero_lower_weights_give_per_slice_2d_streams():
    # with no weight on the lower window the network is the 2-D one on the first 12
    # inputs, so the body is the per-slice 2-D bodies, groups in slice order
    l3 = _layers(H=16, seed=9)
    W0, b0 = l3[0]
    W0 = W0.copy()
    W0[:, 12:] = 0.0
    l3[0] = (W0, b0)
    l2 = [(W0[:, :12].copy(), b0)] + l3[1:]
    vol = synth.mri_volume(4, depth=3, size=20)[:, :14, :]
    G, L = 2, 2
    buf = vo.encode_volume(vol, l3, G, L, ws=1)
    hdr = oracle.parse_header(buf)
    assert (hdr["h"], hdr["w"], hdr["groups"], hdr["k_in"], hdr["n_mix"]) == (42, 20, 6, 21, 0)
    assert hdr["flags"] == 3 | (1 << 12)
    counts, words = [], []
    for z in range(3):
        b2 = sm.encode_image_softmax(vol[z], l2, G, L)
        counts += [len(s) for s in oracle.split_streams(b2, G)]
        words += [np.asarray(s, "<u2").tobytes() for s in oracle.split_streams(b2, G)]
    body = np.asarray(counts, "<u4").tobytes() + b"".join(words)
    assert buf[oracle.HEADER_SIZE:] == body


@pytest.mark.parametrize("ws,G,L", [(0, 1, 4), (1, 2, 2), (2, 3, 1)])
def test_round_trip(ws, G, L):
    layers = _layers(H=16, seed=3 + ws)
    vol = synth.mri_volume(11 + ws, depth=3, size=16)[:, :, :13]
    buf = vo.encode_volume(vol, layers, G, L, ws)
    assert np.array_equal(vo.decode_volume(buf, layers), vol)


def test_length_near_ideal_and_model_check():
    layers = _layers(H=16, seed=21)
    vol = synth.mri_volume(5, depth=2, size=16)
    buf = vo.encode_volume(vol, layers, 1, 2, 1)
    o = sm.deep_forward_bf16(vo.volume_features(vol, 1).reshape(-1, 21), layers)
    ideal = sm.ideal_bits_softmax(o, vol.reshape(-1))
    body_bits = 16 * (len(buf) - oracle.HEADER_SIZE - 4) // 2
    assert ideal <= body_bits <= ideal * 1.02 + 16 * 2 * 2 + 64
    other = _layers(H=16, seed=22)
    with pytest.raises(ValueError):
        vo.decode_volume(buf, other)


def test_twelve_input_network_codes_slices_alone():
    # 12 inputs: each slice's body is its 2-D body; no lag, WS must be 0
    l2 = _layers(H=16, seed=31, k_in=12)
    vol = synth.mri_volume(8, depth=2, size=12)
    buf = vo.encode_volume(vol, l2, 1, 3, 0)
    hdr = oracle.parse_header(buf)
    assert hdr["k_in"] == 12 and hdr["flags"] == 2
    b0, b1 = (sm.encode_image_softmax(vol[z], l2, 1, 3) for z in range(2))
    s0, s1 = oracle.split_streams(b0, 1)[0], oracle.split_streams(b1, 1)[0]
    assert buf[oracle.HEADER_SIZE:] == (np.asarray([len(s0), len(s1)], "<u4").tobytes()
                                        + np.asarray(list(s0) + list(s1), "<u2").tobytes())
    assert np.array_equal(vo.decode_volume(buf, l2), vol)
    assert vo.lag_of(12, 0) == 0 and vo.n_steps_3d(5, 12, 12, 0, k_in=12) == 12 + 33
    with pytest.raises(ValueError):
        vo.encode_volume(vol, l2, 1, 3, 1)
