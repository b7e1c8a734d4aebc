"""Volumes: the 3-D window and the 3-D wavefront (oracle; test infrastructure).

Paper passages followed:
  * Section IV-C (3D Dependencies): the density of a pixel also looks at the
    slice below; a window of two layers (the target's slice and one more).
  * Section IV-C (3D Wavefront), Fig. 6: the 2-D wavefronts of all slices
    run together, each shifted against the one below so that the pixels of
    the lower layer's window are decoded first; with the lower window not
    shifted down (WS = 0) all slices decode at the same time.
  * Section II-B (Neural Network Architecture): the six-layer network with a
    softmax over 256 levels (oracle/softmax.py), here with 21 inputs.

Readings where the paper is silent (the format's choices):
  * window: the 12 causal neighbours of the target's slice (as in 2-D), then
    the 3 x 3 block of the slice below with rows y + WS - 3 .. y + WS - 1 and
    columns x - 1 .. x + 1, row by row; every value scaled to [-1, 1], 0 outside
    the volume (and for the lowest slice);
  * wavefront: pixel (z, y, x) belongs to global step x + 3 y + lag z with
    lag = max(0, 3 WS - 1), the least shift that puts every lower-window pixel
    in an earlier step;
  * stream: the Z slices stacked into one image of Z H rows, coded as a 2-D
    image with Z G groups (G per slice: every group lies in one slice); the
    header's flags hold Z in bits 0..11 and WS in bits 12..15, k_in = 21;
  * a network of 12 inputs codes a volume slice by slice (the window of the
    pixel's own slice only, WS = 0, no lag): the 3-D wavefront without the
    3-D window.

Parity: the window against a brute-force definition and causality (every
lower-window pixel of every voxel is in an earlier step, and one step less of
lag breaks it), the lag against its closed form, the codec by round trips.
"""
from __future__ import annotations

import numpy as np

from .window import NEIGHBOURS, SKEW, scale

K_IN_3D = 21


def lower_offsets(ws: int) -> list:
    """(dy, dx) of the lower slice's 3 x 3 block, row by row."""
    return [(dy, dx) for dy in (ws - 3, ws - 2, ws - 1) for dx in (-1, 0, 1)]


def lag(ws: int) -> int:
    """Steps slice z trails slice z - 1: one more than the largest step offset
    dx + 3 dy of the lower block, at least 0."""
    return max(0, max(dx + SKEW * dy for dy, dx in lower_offsets(ws)) + 1)


def voxel_features(vol, z: int, y: int, x: int, ws: int, depth: int = 8) -> np.ndarray:
    """The 21 scaled window values of voxel (z, y, x), FP64."""
    vol = np.asarray(vol)
    Z, H, W = vol.shape
    out = np.zeros(K_IN_3D, dtype=np.float64)
    for k, (dy, dx) in enumerate(NEIGHBOURS):
        yy, xx = y + dy, x + dx
        if 0 <= yy < H and 0 <= xx < W:
            out[k] = scale(int(vol[z, yy, xx]), depth)
    if z > 0:
        for k, (dy, dx) in enumerate(lower_offsets(ws)):
            yy, xx = y + dy, x + dx
            if 0 <= yy < H and 0 <= xx < W:
                out[12 + k] = scale(int(vol[z - 1, yy, xx]), depth)
    return out


def volume_features(vol, ws: int, depth: int = 8) -> np.ndarray:
    """Features of every voxel, (Z, H, W, 21), vectorised."""
    vol = np.asarray(vol)
    Z, H, W = vol.shape
    s = scale(vol.astype(np.int64), depth)
    out = np.zeros((Z, H, W, K_IN_3D), dtype=np.float64)
    offs = [(0, dy, dx) for dy, dx in NEIGHBOURS] + [(-1, dy, dx) for dy, dx in lower_offsets(ws)]
    for k, (dz, dy, dx) in enumerate(offs):
        src = np.zeros((Z, H, W), dtype=np.float64)
        z0, y0, x0 = max(0, -dz), max(0, -dy), max(0, -dx)
        z1, y1, x1 = Z - max(0, dz), H - max(0, dy), W - max(0, dx)
        if z0 < z1 and y0 < y1 and x0 < x1:
            src[z0:z1, y0:y1, x0:x1] = s[z0 + dz:z1 + dz, y0 + dy:y1 + dy, x0 + dx:x1 + dx]
        out[..., k] = src
    return out


def lag_of(k_in: int, ws: int) -> int:
    """The lag of a network with k_in inputs: none without the slice below."""
    return lag(ws) if k_in == K_IN_3D else 0


def n_steps_3d(Z: int, H: int, W: int, ws: int, k_in: int = K_IN_3D) -> int:
    return W + SKEW * (H - 1) + lag_of(k_in, ws) * (Z - 1)


def _k_in(layers, ws: int) -> int:
    k = int(np.asarray(layers[0][0]).shape[1])
    if k not in (12, K_IN_3D) or (k == 12 and ws != 0):
        raise ValueError("a volume takes 21 inputs, or 12 with WS = 0")
    return k


def volume_flags(Z: int, ws: int) -> int:
    return (Z & 0xFFF) | ((ws & 0xF) << 12)


def cf_volume(vol, layers, ws: int):
    """(c, f) of every voxel by the softmax table rule, in stacked raster order."""
    from .softmax import deep_forward_bf16, net_depth, table_softmax32
    d = net_depth(layers)
    vol = np.asarray(vol, dtype=np.uint8 if d == 8 else np.uint16)
    f = volume_features(vol, ws, d).reshape(-1, K_IN_3D)[:, :_k_in(layers, ws)]
    F = table_softmax32(deep_forward_bf16(f, layers).astype(np.float32))
    v = vol.reshape(-1).astype(np.int64)
    rows = np.arange(v.size)
    return F[rows, v], F[rows, v + 1] - F[rows, v]


def encode_volume(vol, layers, groups: int, lanes: int, ws: int) -> bytes:
    from .container import assemble, pack_header
    from .rans import canonical_order, rans_encode
    from .softmax import header_dtype, net_depth, stored_fingerprint
    d = net_depth(layers)
    vol = np.asarray(vol, dtype=np.uint8 if d == 8 else np.uint16)
    Z, H, W = vol.shape
    c, f = cf_volume(vol, layers, ws)
    streams = []
    for grp in canonical_order(Z * H, W, Z * groups, lanes):
        idx = [y * W + x for (y, x, _) in grp]
        streams.append(rans_encode([(c[i], f[i]) for i in idx], [ln for (_, _, ln) in grp], lanes))
    Hn = np.asarray(layers[0][0]).shape[0]
    hdr = pack_header(Z * H, W, Z * groups, lanes, dtype=header_dtype(d), h1=Hn, h2=Hn, n_mix=0,
                      k_in=_k_in(layers, ws),
                      fp=stored_fingerprint(layers), flags=volume_flags(Z, ws))
    return assemble(hdr, streams)


def decode_volume(buf: bytes, layers) -> np.ndarray:
    from .container import parse_header, split_streams
    from .rans import canonical_order, rans_decode
    from .softmax import (deep_forward_bf16, header_dtype, net_depth, stored_fingerprint,
                          table_softmax32)
    hdr = parse_header(buf)
    Z, ws = hdr["flags"] & 0xFFF, hdr["flags"] >> 12
    k_in = _k_in(layers, ws)
    d = net_depth(layers)
    if (hdr["n_mix"] != 0 or hdr["k_in"] != k_in or hdr["dtype"] != header_dtype(d)
            or hdr["fingerprint"] != stored_fingerprint(layers)):
        raise ValueError("stream was coded with another model")
    H, W = hdr["h"] // Z, hdr["w"]
    G, lanes = hdr["groups"] // Z, hdr["lanes"]
    vol = np.zeros((Z, H, W), dtype=np.uint8 if d == 8 else np.uint16)
    streams = split_streams(buf, Z * G)
    # a slice's windows reach only the slice below: slices in order, groups in order
    for grp, words in zip(canonical_order(Z * H, W, Z * G, lanes), streams):
        def find(i, slot, grp=grp):
            yt, x, _ = grp[i]
            z, y = divmod(yt, H)
            o = deep_forward_bf16(voxel_features(vol, z, y, x, ws, d)[None, :k_in], layers)
            F = table_softmax32(o.astype(np.float32))[0]
            v = int(np.searchsorted(F, slot, side="right")) - 1
            vol[z, y, x] = v
            return v, int(F[v]), int(F[v + 1] - F[v])
        _, ok = rans_decode(words, lanes, [ln for (_, _, ln) in grp], find)
        if not ok:
            raise ValueError("corrupt stream")
    return vol
