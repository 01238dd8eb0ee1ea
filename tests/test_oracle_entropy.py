"""Pins of the entropy-stage oracle (order-0 Huffman over stream bytes).

The code lengths are checked against a textbook example with a unique
optimum, exhaustive search over small alphabets, Kraft's equality and the
entropy bound; the canonical codes against the worked example of RFC 1951
Sec. 3.2.2; the bit layout by an independent decoder written here; and the
whole coder by round trips (empty, one value, all 256 values, skewed data, a
CHR stream).
"""
import itertools

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.filterwarnings("ignore")


def _hist(counts):
    h = np.zeros(256, np.uint64)
    for s, c in counts.items():
        h[s] = c
    return h


def test_textbook_example_lengths():
    # a unique optimum: frequencies 45, 13, 12, 16, 9, 5 give lengths 1, 3, 3, 3, 4, 4
    f = {0: 45, 1: 13, 2: 12, 3: 16, 4: 9, 5: 5}
    ln = oracle.huff_lengths(_hist(f))
    assert [int(ln[s]) for s in range(6)] == [1, 3, 3, 3, 4, 4]
    assert not ln[6:].any()


def test_rfc1951_canonical_codes():
    # RFC 1951 Sec. 3.2.2: lengths (3, 3, 3, 3, 3, 2, 4, 4) for A..H give
    # 010, 011, 100, 101, 110, 00, 1110, 1111
    ln = np.zeros(256, np.uint8)
    ln[:8] = [3, 3, 3, 3, 3, 2, 4, 4]
    c = oracle.huff_codes(ln)
    assert [format(int(c[s]), f"0{int(ln[s])}b") for s in range(8)] == \
        ["010", "011", "100", "101", "110", "00", "1110", "1111"]


def _kraft(ln):
    return sum(2.0 ** -int(v) for v in ln if v)


def _best_cost(freqs):
    """Minimum sum f*l over all length vectors satisfying Kraft's inequality."""
    m = len(freqs)
    best = None
    for ls in itertools.product(range(1, m + 1), repeat=m):
        if sum(2.0 ** -l for l in ls) <= 1.0 + 1e-12:
            c = sum(f * l for f, l in zip(freqs, ls))
            best = c if best is None else min(best, c)
    return best


@pytest.mark.parametrize("seed", range(12))
def test_lengths_are_optimal_on_small_alphabets(seed):
    rng = np.random.default_rng(seed)
    m = int(rng.integers(2, 7))
    freqs = [int(v) for v in rng.integers(1, 50, m)]
    syms = rng.choice(256, m, replace=False)
    ln = oracle.huff_lengths(_hist(dict(zip(syms, freqs))))
    got = sum(f * int(ln[s]) for f, s in zip(freqs, syms))
    assert got == _best_cost(freqs)
    assert abs(_kraft(ln) - 1.0) < 1e-12


@pytest.mark.parametrize("seed", range(8))
def test_kraft_equality_and_entropy_bound(seed):
    rng = np.random.default_rng(100 + seed)
    h = rng.geometric(0.05, 256).astype(np.uint64) * (rng.random(256) < 0.7)
    ln = oracle.huff_lengths(h)
    assert abs(_kraft(ln[h > 0]) - 1.0) < 1e-12
    assert not ln[h == 0].any()
    p = h[h > 0] / h.sum()
    H = -(p * np.log2(p)).sum()
    avg = (h * ln).sum() / h.sum()
    assert H - 1e-12 <= avg < H + 1.0


def test_length_limit_on_deep_trees():
    # Fibonacci counts make a Huffman tree as deep as there are symbols
    fib = [1, 1]
    while len(fib) < 30:
        fib.append(fib[-1] + fib[-2])
    h = _hist({s: c for s, c in enumerate(fib)})
    for maxlen in (12, 15, 20):
        ln = oracle.huff_lengths(h, maxlen=maxlen)
        assert int(ln.max()) == maxlen
        assert abs(_kraft(ln) - 1.0) < 1e-12
        # more frequent values never get longer codes
        order = np.argsort(-np.array(fib), kind="stable")
        assert np.all(np.diff([int(ln[s]) for s in order]) >= 0)


def test_single_and_no_values():
    ln = oracle.huff_lengths(_hist({7: 10}))
    assert int(ln[7]) == 1 and int(ln.sum()) == 1
    assert not oracle.huff_lengths(np.zeros(256, np.uint64)).any()


def _decode_here(enc):
    """An independent decoder of the format (bit by bit from the table of codes)."""
    u32 = lambda o: int.from_bytes(bytes(enc[o:o + 4]), "little")
    n = int.from_bytes(bytes(enc[8:16]), "little")
    chunk, nch, maxlen = u32(16), u32(20), u32(32)
    ln = enc[64:320]
    codes = oracle.huff_codes(ln)
    table = {(int(ln[s]), int(codes[s])): s for s in range(256) if ln[s]}
    base = ((320 + 4 * (nch + 1)) + 7) // 8 * 8
    out = []
    for c in range(nch):
        bit = 32 * u32(320 + 4 * c)
        for _ in range(min(chunk, n - c * chunk)):
            v, l = 0, 0
            while (l, v) not in table:
                v = (v << 1) | ((int(enc[base + bit // 8]) >> (bit % 8)) & 1)
                bit += 1
                l += 1
                assert l <= maxlen
            out.append(table[(l, v)])
    return np.array(out, np.uint8)


def test_bit_layout_by_an_independent_decoder():
    rng = np.random.default_rng(5)
    d = np.minimum(rng.geometric(0.3, 3000), 40).astype(np.uint8)
    enc = oracle.entropy_encode(d, chunk=512)
    assert np.array_equal(_decode_here(enc), d)


@pytest.mark.parametrize("kind", ["empty", "one", "same", "all256", "skewed", "ragged"])
def test_round_trips(kind):
    rng = np.random.default_rng(9)
    d = {"empty": np.zeros(0, np.uint8),
         "one": np.array([200], np.uint8),
         "same": np.full(5000, 17, np.uint8),
         "all256": np.tile(np.arange(256, dtype=np.uint8), 9),
         "skewed": np.minimum(rng.geometric(0.2, 70000), 255).astype(np.uint8),
         "ragged": rng.integers(0, 256, 512 * 7 + 13).astype(np.uint8)}[kind]
    enc = oracle.entropy_encode(d)
    assert int.from_bytes(bytes(enc[0:4]), "little") == 0x48524843
    assert int.from_bytes(bytes(enc[8:16]), "little") == d.size
    assert int.from_bytes(bytes(enc[24:32]), "little") == enc.size
    assert np.array_equal(oracle.entropy_decode(enc), d)
    if kind == "same":
        # one value: one bit per byte
        assert enc.size < 5000 // 8 + 400


def test_round_trip_of_a_chr_stream_and_its_gain():
    f = np.random.default_rng(2).standard_normal((40, 37, 70)).astype(np.float32)
    s = oracle.compress(f, 0.05, [0.0], levels=3, block=16)["stream"]
    enc = oracle.entropy_encode(s)
    assert np.array_equal(oracle.entropy_decode(enc), s)
    # never worse than the order-0 bound by more than 1 bit per byte plus the tables
    cnt = np.bincount(s, minlength=256).astype(np.float64)
    p = cnt[cnt > 0] / cnt.sum()
    H = -(p * np.log2(p)).sum()
    assert enc.size * 8 <= (H + 1) * s.size + 8 * (320 + 4 * (s.size // 512 + 2) + 4 * (s.size // 512 + 1) + 8)
