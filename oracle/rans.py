"""Interleaved rANS with 32-bit state, and the lane / order layout
(oracle; test infrastructure).

Paper passages followed:
  * Section II-B (rANS): the range variant of Duda's asymmetric numeral
    systems; because the wavefront codes several pixels at once, several
    coder instances run in parallel and write several bitstreams, at most
    one per pixel row; the GPU coder uses 32-bit arithmetic.
  * Section II-B (Preprocessor): the wavefront order (step t = x + 3y here).

Textbook rANS (Duda 2013; the byte-wise form of Giesen 2014) with
probability scale M = 2^16, state interval [2^16, 2^32) and 16-bit
renormalisation words:
  encode symbol (c, f):  if x >= f * 2^16: emit x & 0xFFFF, x >>= 16
                         x = (x // f) * 2^16 + (x % f) + c
  decode:                slot = x & 0xFFFF; find s with c_s <= slot < c_s + f_s
                         x = f_s * (x >> 16) + slot - c_s
                         if x < 2^16: x = (x << 16) | next word

Layout readings (the paper fixes none of this), all explicit in the arguments:
  * G groups, each coding S row strips (S = 1 by default).  The image is cut
    into S*G strips, strip b owning rows [floor(bH/(SG)), floor((b+1)H/(SG)));
    group g codes strips g, G + g, ..., (S-1)G + g, spread over the image, so
    that when a strip is shorter than the wavefront's band of active rows a
    group has rows in fewer steps at once.  One stream per group, shared by
    its L lanes (interleaved rANS).
  * Row y of a strip starting at row r belongs to lane (y - r) mod L, block
    j = (y - r) div L.
  * Canonical order in a group: its strips in ascending order, each strip in
    ascending (t = x + 3y, j, lane); a lane's state carries from one strip to
    the next.  Encoding walks it backwards; every lane starts at 2^16; after the last symbol
    the lanes' states are appended (for lanes L-1..0: high half, then low
    half) and the whole push sequence is reversed, so a stream read forward
    starts with the L states as (low, high) 16-bit pairs for lanes 0..L-1,
    followed by the renormalisation words in decoding order.

Parity: pinned by a hand-computed one-lane stream (tests/golden), the
closed-form byte shuffle of the uniform table, the one-word-per-symbol
case f = 1, final decoder states equal to 2^16, and round trips.
"""
from __future__ import annotations

from .window import SKEW

RANS_L = 1 << 16
WORD_BITS = 16
PROB_BITS = 16


def group_rows(h: int, groups: int) -> list:
    """Row boundaries r_0..r_G of G row strips of near-equal height."""
    return [(g * h) // groups for g in range(groups + 1)]


def group_strips(groups: int, strips: int, g: int) -> list:
    """Indices of the strips group g codes, in its coding order."""
    return [s * groups + g for s in range(strips)]


def _strip_order(y0: int, y1: int, w: int, lanes: int, skew: int) -> list:
    items = []
    for y in range(y0, y1):
        r = y - y0
        lane, blk = r % lanes, r // lanes
        for x in range(w):
            items.append((x + skew * y, blk, lane, y, x))
    items.sort()
    return [(it[3], it[4], it[2]) for it in items]


def canonical_order(h: int, w: int, groups: int, lanes: int, skew: int = SKEW, only=None,
                    strips: int = 1) -> list:
    """For each group, the list of (y, x, lane) in canonical order.

    only: optional set of group indices to build (others are left empty).
    strips: row strips per group (S above).
    """
    rows = group_rows(h, groups * strips)
    out = []
    for g in range(groups):
        if only is not None and g not in only:
            out.append([])
            continue
        seq = []
        for b in group_strips(groups, strips, g):
            seq += _strip_order(rows[b], rows[b + 1], w, lanes, skew)
        out.append(seq)
    return out


def rans_encode(cf, lanes_seq, n_lanes: int) -> list:
    """Encode one group's symbols.

    cf: sequence of (c, f) in canonical order; lanes_seq: the lane of each
    symbol.  Returns the stream as a list of 16-bit words in reading order.
    """
    x = [RANS_L] * n_lanes
    pushes = []
    for i in range(len(cf) - 1, -1, -1):
        c, f = int(cf[i][0]), int(cf[i][1])
        lane = int(lanes_seq[i])
        assert 1 <= f and 0 <= c and c + f <= (1 << PROB_BITS)
        s = x[lane]
        if s >= (f << PROB_BITS):
            pushes.append(s & 0xFFFF)
            s >>= WORD_BITS
        s = ((s // f) << PROB_BITS) + (s % f) + c
        assert RANS_L <= s < (1 << 32)
        x[lane] = s
    for lane in range(n_lanes - 1, -1, -1):
        pushes.append(x[lane] >> 16)
        pushes.append(x[lane] & 0xFFFF)
    return pushes[::-1]


class RansDecoder:
    """One group's stream, decoded one symbol at a time in canonical order.

    Decoding can pause between symbols, so that a caller may interleave the
    groups in any order the symbols' dependencies allow (strips of one group
    depend on strips of other groups).
    """

    def __init__(self, words, n_lanes: int):
        self.words = words
        self.n = len(words)
        self.ok = self.n >= 2 * n_lanes
        self.x = ([words[2 * l] | (words[2 * l + 1] << 16) for l in range(n_lanes)]
                  if self.ok else [RANS_L] * n_lanes)
        self.pos = 2 * n_lanes

    def decode(self, lane: int, find):
        """find(slot) -> (symbol, c, f); returns the symbol."""
        s = self.x[lane]
        slot = s & 0xFFFF
        sym, c, f = find(slot)
        s = f * (s >> 16) + slot - c
        if s < RANS_L:
            if self.pos < self.n:
                s = (s << 16) | self.words[self.pos]
            else:
                self.ok = False
                s = s << 16
            self.pos += 1
        self.x[lane] = s
        return sym

    def finished(self) -> bool:
        """Every lane back at 2^16, every word consumed, no read past the end."""
        return self.ok and self.pos == self.n and all(v == RANS_L for v in self.x)


def rans_decode(words, n_lanes: int, lanes_seq, find):
    """Decode one group's symbols in canonical order.

    find(i, slot) -> (symbol, c, f) locates the symbol of the i-th position
    whose interval [c, c+f) contains slot; it may depend on symbols already
    decoded.  Returns (symbols, ok) where ok means every lane ended at 2^16,
    every word was consumed and no read ran past the end.
    """
    if len(words) < 2 * n_lanes:
        return [], False
    dec = RansDecoder(words, n_lanes)
    out = [dec.decode(lane, lambda slot, i=i: find(i, slot)) for i, lane in enumerate(lanes_seq)]
    return out, dec.finished()
