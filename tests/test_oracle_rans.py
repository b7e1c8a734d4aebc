"""Pins of the oracle's interleaved rANS (CPU)."""
import numpy as np

import oracle
import synth


def _case(lines, tag):
    rows = [ln.split()[1:] for ln in lines if ln.startswith(tag + " ")]
    lanes = int([r for r in rows if r[0] == "lanes"][0][1])
    syms = [tuple(int(v) for v in r[1:]) for r in rows if r[0] == "sym"]
    words = [int(v) for v in [r for r in rows if r[0] == "words"][0][1:]]
    byts = [r for r in rows if r[0] == "bytes"]
    return lanes, syms, words, (bytes.fromhex(byts[0][1]) if byts else None)


def test_hand_computed_streams(golden):
    lines = golden("rans_hand.txt")
    for tag in ("caseA", "caseB"):
        lanes, syms, words, raw = _case(lines, tag)
        got = oracle.rans_encode([(c, f) for (_, c, f) in syms], [l for (l, _, _) in syms], lanes)
        assert got == words, tag
        if raw is not None:
            assert np.asarray(got, dtype="<u2").tobytes() == raw

        def find(i, slot):
            _, c, f = syms[i]
            assert c <= slot < c + f
            return i, c, f
        out, ok = oracle.rans_decode(words, lanes, [l for (l, _, _) in syms], find)
        assert ok and out == list(range(len(syms)))


def test_uniform_table_closed_forms():
    # f = 256, c = 256 v turns one encode step into x' = ((x >> 8) << 16) | (v << 8) | (x & 0xFF).
    # From x = 2^16 this gives, for 1, 2 and 3 symbols (decoding order):
    #   [v0<<8, 256] ; [v0<<8, 1, v1<<8] ; [v0<<8, 256+v1, v2<<8]
    for v0, v1, v2 in ((0, 0, 0), (255, 1, 128), (17, 200, 3)):
        enc = lambda vs: oracle.rans_encode([(256 * v, 256) for v in vs], [0] * len(vs), 1)
        assert enc([v0]) == [v0 << 8, 256]
        assert enc([v0, v1]) == [v0 << 8, 1, v1 << 8]
        assert enc([v0, v1, v2]) == [v0 << 8, 256 + v1, v2 << 8]


def test_unit_frequency_costs_one_word_each():
    rng = np.random.default_rng(0)
    n, lanes = 500, 7
    c = rng.integers(0, 1 << 16, size=n)
    ln = rng.integers(0, lanes, size=n)
    words = oracle.rans_encode([(int(x), 1) for x in c], ln, lanes)
    assert len(words) == n + 2 * lanes


def _random_group(seed, n, lanes, n_tab=40):
    tabs = synth.random_tables(n_tab, seed).astype(np.int64)
    rng = np.random.default_rng(seed + 1)
    tid = rng.integers(0, n_tab, size=n)
    sym = synth.random_symbols_from_tables(tabs, tid, seed + 2)
    ln = rng.integers(0, lanes, size=n)
    cf = [(tabs[t, s], tabs[t, s + 1] - tabs[t, s]) for t, s in zip(tid, sym.astype(np.int64))]
    return tabs, tid, sym, ln, cf


def test_random_round_trip_and_final_states():
    for seed, n, lanes in ((0, 3000, 32), (1, 1, 32), (2, 777, 5), (3, 0, 3)):
        tabs, tid, sym, ln, cf = _random_group(seed, n, lanes)
        words = oracle.rans_encode(cf, ln, lanes)

        def find(i, slot):
            F = tabs[tid[i]]
            v = int(np.searchsorted(F, slot, side="right")) - 1
            return v, int(F[v]), int(F[v + 1] - F[v])
        out, ok = oracle.rans_decode(words, lanes, ln, find)
        assert ok and np.array_equal(np.asarray(out, dtype=np.int64), sym.astype(np.int64))
        # Per lane, 16 * renormalisation words + log2(final state) - 16 equals the symbols'
        # cost plus the state rounding r (|r| <= 0.02 bit per symbol here); the final state
        # lies in [2^16, 2^32) and is flushed as two words.  So the stream holds between
        # cost + 16 * lanes and cost + 32 * lanes bits, give or take r.
        cost = sum(-np.log2(f / 65536.0) for (_, f) in cf)
        bits = 16 * len(words)
        slack = 0.02 * n + 1
        assert cost + 16 * lanes - slack <= bits <= cost + 32 * lanes + slack


def test_corruption_is_detected():
    tabs, tid, sym, ln, cf = _random_group(5, 2000, 32)
    words = oracle.rans_encode(cf, ln, 32)

    def find(i, slot):
        F = tabs[tid[i]]
        v = int(np.searchsorted(F, slot, side="right")) - 1
        return v, int(F[v]), int(F[v + 1] - F[v])
    bad = list(words); bad[len(bad) // 2] ^= 0x1234
    out, ok = oracle.rans_decode(bad, 32, ln, find)
    assert not ok or out != list(sym)
    out, ok = oracle.rans_decode(words[:-1], 32, ln, find)
    assert not ok


def test_canonical_order_layout():
    order = oracle.canonical_order(70, 9, 2, 32)
    rows = oracle.group_rows(70, 2)
    assert rows == [0, 35, 70]
    seen = set()
    for g, grp in enumerate(order):
        keys = []
        for (y, x, lane) in grp:
            assert rows[g] <= y < rows[g + 1]
            assert lane == (y - rows[g]) % 32
            keys.append((x + 3 * y, (y - rows[g]) // 32, lane))
            seen.add((y, x))
        assert keys == sorted(keys) and len(set(keys)) == len(keys)
    assert len(seen) == 70 * 9
