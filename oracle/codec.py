"""Whole-image encode and decode (oracle; test infrastructure).

Paper passages followed:
  * Section II-A and Fig. 2: encoding passes each pixel's window through
    the network and codes the pixel with the resulting PDF; decoding runs
    the same window through the same network, decodes the pixel from the
    coder state, and the pixel then joins later windows.
  * Section II-B (Preprocessor): wavefront parallelism, identical network
    inputs on both sides.
  * Section II-B (rANS): multiple coder instances and bitstreams.

The oracle encodes in two plain passes: every pixel's (c, f) from the whole
image (the network applied to the matrix of all windows), then each group's
rANS walk.  Decoding goes pixel by pixel in canonical order, evaluating the
network on windows of the partially decoded image, which is the paper's
decoder without its parallelism.  Strips are decoded in ascending order, each
continuing its group's coder state: a strip's windows reach only into rows of
earlier strips and into its own earlier canonical positions.

Parity: pinned by oracle round trips (decode(encode(x)) == x) and by the
coded length against the ideal code length.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .container import (pack_header, parse_header, assemble, split_streams, fingerprint,
                        image_flags, image_strips)
from .freq import table_levels32, table_full32
from .network import mlp_forward, mixture_head
from .rans import RansDecoder, canonical_order, group_rows, group_strips, rans_encode
from .window import causal_features, pixel_features


@dataclass(frozen=True)
class OracleCoder:
    groups: int = 1
    lanes: int = 32
    strips: int = 1  # row strips per group


def weights_fingerprint(weights) -> int:
    return fingerprint([weights[k] for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def _mlp(weights, feats):
    return mlp_forward(feats, weights["W1"], weights["b1"], weights["W2"], weights["b2"],
                       weights["W3"], weights["b3"])


def params32_for_image(img, weights):
    """FP32 roundings of the FP64 mixture parameters of every pixel, raster order."""
    pi, mu, inv_s = mixture_head(_mlp(weights, causal_features(img)))
    return pi.astype(np.float32), mu.astype(np.float32), inv_s.astype(np.float32)


def cf_for_image(img, weights):
    """(c, f) of every pixel's actual value by the FP32 table rule, raster order."""
    pi, mu, is_ = params32_for_image(img, weights)
    v = np.asarray(img, dtype=np.int64).ravel()
    F = table_levels32(np.stack([v, v + 1], axis=1), pi, mu, is_)
    return F[:, 0], F[:, 1] - F[:, 0]


def encode_image(img, weights, coder: OracleCoder) -> bytes:
    img = np.asarray(img, dtype=np.uint8)
    h, w = img.shape
    c, f = cf_for_image(img, weights)
    streams = []
    for grp in canonical_order(h, w, coder.groups, coder.lanes, strips=coder.strips):
        idx = [y * w + x for (y, x, _) in grp]
        streams.append(rans_encode([(c[i], f[i]) for i in idx],
                                   [lane for (_, _, lane) in grp], coder.lanes))
    hdr = pack_header(h, w, coder.groups, coder.lanes, dtype=0,
                      h1=weights["W1"].shape[0], h2=weights["W2"].shape[0],
                      fp=weights_fingerprint(weights), flags=image_flags(coder.strips))
    return assemble(hdr, streams)


def decode_image(buf: bytes, weights) -> np.ndarray:
    hdr = parse_header(buf)
    if hdr["fingerprint"] != weights_fingerprint(weights):
        raise ValueError("stream was coded with another model")
    h, w, groups, lanes = hdr["h"], hdr["w"], hdr["groups"], hdr["lanes"]
    strips = image_strips(hdr["flags"])
    streams = split_streams(buf, groups)
    img = np.zeros((h, w), dtype=np.uint8)
    order = canonical_order(h, w, groups, lanes, strips=strips)
    decs = [RansDecoder(words, lanes) for words in streams]
    if any(len(words) < 2 * lanes for words in streams):
        raise ValueError("corrupt stream")
    rows = group_rows(h, groups * strips)
    done = [0] * groups  # canonical positions decoded per group
    for s in range(strips):
        for g in range(groups):
            b = group_strips(groups, strips, g)[s]
            n = (rows[b + 1] - rows[b]) * w
            for y, x, lane in order[g][done[g]:done[g] + n]:
                def find(slot, y=y, x=x):
                    o = _mlp(weights, pixel_features(img, y, x)[None, :])
                    pi, mu, inv_s = mixture_head(o)
                    F = table_full32(pi.astype(np.float32), mu.astype(np.float32),
                                     inv_s.astype(np.float32))[0]
                    v = int(np.searchsorted(F, slot, side="right")) - 1
                    img[y, x] = v
                    return v, int(F[v]), int(F[v + 1] - F[v])
                decs[g].decode(lane, find)
            done[g] += n
    if not all(d.finished() for d in decs):
        raise ValueError("corrupt stream")
    return img
