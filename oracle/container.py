"""Bitstream container (oracle; test infrastructure).

Paper passages followed:
  * Section II-B (rANS): several coder instances write several bitstreams.
  * Section II-B (Preprocessor): the network weights are part of the codec
    (encoder and decoder must evaluate the same network), not of the stream.
  * Section III-A: rates are quoted excluding header information.

The paper defines no container.  Our reading, little-endian:
  36-byte header  "DLIC" | u16 version=1 | u16 flags=0 | u32 H | u32 W |
                  u8 k_in=12 | u8 n_mix=5 | u8 dtype | u8 skew=3 |
                  u16 h1 | u16 h2 | u8 prob_bits=16 | u8 lanes per group |
                  u16 G | u64 model fingerprint
  G x u32         16-bit word count of each group's stream (flush included)
  G streams       each as little-endian 16-bit words, in group order.
The model fingerprint is 64-bit FNV-1a over the little-endian bytes of
W1, b1, W2, b2, W3, b3 in that order, as stored.
flags: a volume stores its slice count Z (1..4095) in bits 0..11 and its
window shift in bits 12..15; an image has bits 0..11 zero and stores S - 1,
S the row strips per group (1..16), in bits 12..15.

Parity: pinned by round trips of header fields and by the published FNV-1a
test vectors.
"""
from __future__ import annotations

import struct

import numpy as np

HEADER_FMT = "<4sHHIIBBBBHHBBHQ"
HEADER_SIZE = struct.calcsize(HEADER_FMT)
MAGIC = b"DLIC"
VERSION = 1

FNV_OFFSET = 0xCBF29CE484222325
FNV_PRIME = 0x100000001B3


def fingerprint(arrays) -> int:
    """64-bit FNV-1a over the bytes of the given arrays, concatenated."""
    h = FNV_OFFSET
    for a in arrays:
        for byte in np.ascontiguousarray(a).tobytes():
            h ^= byte
            h = (h * FNV_PRIME) & 0xFFFFFFFFFFFFFFFF
    return h


def pack_header(h, w, groups, lanes, dtype=0, h1=0, h2=0, fp=0, k_in=12, n_mix=5,
                skew=3, prob_bits=16, flags=0) -> bytes:
    return struct.pack(HEADER_FMT, MAGIC, VERSION, flags, h, w, k_in, n_mix, dtype, skew,
                       h1, h2, prob_bits, lanes, groups, fp)


def parse_header(buf: bytes) -> dict:
    if len(buf) < HEADER_SIZE:
        raise ValueError("stream shorter than the header")
    f = struct.unpack(HEADER_FMT, bytes(buf[:HEADER_SIZE]))
    if f[0] != MAGIC or f[1] != VERSION:
        raise ValueError("not a DLIC v1 stream")
    keys = ("magic", "version", "flags", "h", "w", "k_in", "n_mix", "dtype", "skew",
            "h1", "h2", "prob_bits", "lanes", "groups", "fingerprint")
    return dict(zip(keys, f))


def image_flags(strips: int) -> int:
    """The flags field of an image coded with `strips` row strips per group."""
    if not 1 <= strips <= 16:
        raise ValueError("1..16 strips per group")
    return (strips - 1) << 12


def image_strips(flags: int) -> int:
    """Row strips per group of an image stream; raises for a volume's flags."""
    if flags & 0xFFF:
        raise ValueError("a volume stream, not an image")
    return (flags >> 12) + 1


def assemble(header: bytes, streams) -> bytes:
    """Header, the per-group word counts, then every group's words."""
    counts = struct.pack("<%dI" % len(streams), *[len(s) for s in streams])
    body = b"".join(np.asarray(s, dtype="<u2").tobytes() for s in streams)
    return header + counts + body


def split_streams(buf: bytes, groups: int) -> list:
    """Per-group word lists from a whole stream; raises on inconsistent sizes."""
    off = HEADER_SIZE
    if len(buf) < off + 4 * groups:
        raise ValueError("stream truncated in the word-count table")
    counts = struct.unpack_from("<%dI" % groups, buf, off)
    off += 4 * groups
    if len(buf) != off + 2 * sum(counts):
        raise ValueError("stream length does not match its word counts")
    out = []
    for n in counts:
        out.append(np.frombuffer(buf, dtype="<u2", count=n, offset=off).astype(np.int64).tolist())
        off += 2 * n
    return out
