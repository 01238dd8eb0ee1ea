"""Pins of block merging before compression (Sec. II.A, third step of CHR
generation: blocks merged into larger rectangular grids so that they are
compressed and visualized more efficiently).

The paper gives no merging rule.  The reading pinned here: a block's index
signature is the set of candidate isovalues its input range crosses
(min < k <= max over the closed extent); blocks of equal signature are
merged greedily, in lexicographic block order, into rectangular units of at
most `merge` blocks per axis (grown along x, then y, then z), and each unit
is stored as one closed extent.  The hierarchy is global, so codes and the
reconstruction are those of the unmerged stream; only the grouping of points
into sections changes, and points on faces between merged blocks are stored
once instead of twice.

Pins: units derived by hand for two block patterns, equality of codes,
flags and every level's reconstruction with the unmerged stream, byte
equality with the plain stream when merging is off, a smaller stream when
blocks merge, the tiling check of the reader, argument errors, and the
extraction-side box over merged units.
"""
import struct

import numpy as np
import pytest

import oracle
from paper_2408_05462_amd import inputs
from test_stream_layout import Stream, _checksum


def _units(stream):
    S = Stream(stream)
    return [tuple(S.box(b)[0]) + tuple(S.box(b)[1]) for b in range(S.nblocks)]


def test_units_without_candidates_by_hand():
    """No candidate isovalues: every block has the empty signature, so a
    3 x 3 x 3 block grid with merge = 2 splits into 8 units, derived by hand
    from the growth order (x, then y, then z)."""
    f = np.random.default_rng(0).standard_normal((11, 12, 10)).astype(np.float32)
    r = oracle.compress(f, 0.05, [], levels=3, block=4, merge=2)
    assert _units(r["stream"]) == [
        (0, 0, 0, 2, 2, 2), (0, 0, 2, 2, 2, 3), (0, 2, 0, 2, 3, 2), (0, 2, 2, 2, 3, 3),
        (2, 0, 0, 3, 2, 2), (2, 0, 2, 3, 2, 3), (2, 2, 0, 3, 3, 2), (2, 2, 2, 3, 3, 3),
    ]
    info = oracle.stream_info(r["stream"])
    assert info.nblocks == 8 and info.merge == 2 and list(info.mb) == [2, 2, 2] and info.flags == 8


# block grid 2 x 3 x 4 (z, y, x); 1 marks blocks whose input crosses k = 0.5
PATTERN = np.array([
    [[1, 1, 0, 0], [1, 1, 0, 1], [0, 0, 0, 1]],
    [[1, 1, 0, 0], [1, 1, 1, 1], [0, 0, 0, 1]],
])


def test_units_of_a_signature_pattern_by_hand():
    """2.0 everywhere, 0.0 at the centre point of the marked blocks (a point
    no other closed extent holds), candidate 0.5: exactly the marked blocks
    cross it.  With merge = 4 the greedy rule gives these 7 units."""
    B = 4
    f = np.full((9, 13, 17), 2.0, np.float32)
    for z, y, x in zip(*np.nonzero(PATTERN)):
        f[B * z + 2, B * y + 2, B * x + 2] = 0.0
    r = oracle.compress(f, 0.01, [0.5], levels=3, block=B, merge=4)
    assert _units(r["stream"]) == [
        (0, 0, 0, 2, 2, 2),   # the marked 2 x 2 x 2 corner
        (0, 0, 2, 2, 1, 4),   # unmarked, grown along x and z, not y
        (0, 1, 2, 1, 3, 3),   # unmarked, stopped by a marked block along x and z
        (0, 1, 3, 2, 3, 4),   # marked column along y and z
        (0, 2, 0, 2, 3, 2),   # unmarked, stopped by unit 2 along x
        (1, 1, 2, 2, 2, 3),   # marked single block
        (1, 2, 2, 2, 3, 3),   # unmarked single block
    ]
    # merged units keep the index exact for the candidate: a unit crosses
    # 0.5 iff its blocks do
    S = Stream(r["stream"])
    for b in range(S.nblocks):
        b0, b1 = S.box(b)
        mn, mx = S.f32(S.payload - 48 * S.nblocks + 16 * b), S.f32(S.payload - 48 * S.nblocks + 16 * b + 4)
        assert (mn < 0.5 <= mx) == bool(PATTERN[b0[0], b0[1], b0[2]])


MERGE_CASES = [
    ("smooth", (40, 37, 45), 3, 8, 2, [0.25, 0.5]),
    ("grf", (33, 35, 31), 4, 8, 3, [0.0]),
    ("normal", (21, 19, 23), 2, 4, 4, [0.0, 1.0]),
    ("smooth", (1, 30, 70), 2, 8, 3, [0.5]),
]


def _field(kind, shape):
    if kind == "normal":
        return np.random.default_rng(7).standard_normal(shape).astype(np.float32)
    n = max(shape)
    if kind == "grf":
        return np.ascontiguousarray(inputs.grf(n, 0.4)[: shape[0], : shape[1], : shape[2]])
    return np.ascontiguousarray(inputs.gaussians(n, seed=5)[: shape[0], : shape[1], : shape[2]])


@pytest.mark.parametrize("case", MERGE_CASES, ids=lambda c: f"{c[0]}-{'x'.join(map(str, c[1]))}-M{c[4]}")
def test_merging_keeps_codes_and_reconstruction(case):
    kind, shape, nL, B, M, isos = case
    f = _field(kind, shape)
    e = inputs.abs_error_bound(1e-3, f)
    plain = oracle.compress(f, e, isos, levels=nL, block=B)
    merged = oracle.compress(f, e, isos, levels=nL, block=B, merge=M)
    for key in ("q", "flags", "xr"):
        assert np.array_equal(plain[key], merged[key]), key
    q, ex = oracle.stream_codes(merged["stream"])
    assert np.array_equal(q, plain["q"]) and np.array_equal(ex, plain["flags"] != 0)
    for lv in range(nL):
        a = oracle.decompress(plain["stream"], lv)
        b = oracle.decompress(merged["stream"], lv)
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32)), lv
    assert oracle.stream_verify(merged["stream"]) == 0
    pi, mi = oracle.stream_info(plain["stream"]), oracle.stream_info(merged["stream"])
    assert (mi.n_outlier, mi.n_corrected) == (pi.n_outlier, pi.n_corrected)
    if mi.nblocks < pi.nblocks:
        # fewer sections and no duplicated faces inside a unit
        assert len(merged["stream"]) < len(plain["stream"])


def test_merge_off_is_the_plain_stream():
    f = _field("smooth", (30, 31, 29))
    plain = oracle.compress(f, 1e-3, [0.5], levels=3, block=8)
    for m in (0, 1):
        r = oracle.compress(f, 1e-3, [0.5], levels=3, block=8, merge=m)
        assert r["stream"].tobytes() == plain["stream"].tobytes()


def test_merged_stream_size_counts_shared_faces_once():
    """Constant-code field: every point codes to 0, so a section holds its
    points' chunk headers and nothing else; the merged stream stores each
    face point shared by two blocks of a unit once."""
    f = np.zeros((17, 17, 17), np.float32)
    plain = oracle.compress(f, 0.1, [], levels=2, block=8)
    merged = oracle.compress(f, 0.1, [], levels=2, block=8, merge=2)
    assert oracle.stream_info(merged["stream"]).nblocks == 1
    S = Stream(merged["stream"])
    npts = sum(struct.unpack_from("<I", S.s, S.section(0, lv)[0])[0] for lv in range(2))
    assert npts == 17 ** 3
    Sp = Stream(plain["stream"])
    npts_plain = sum(struct.unpack_from("<I", Sp.s, Sp.section(b, lv)[0])[0] for b in range(8) for lv in range(2))
    assert npts_plain == 8 * 9 ** 3


def _resum(s):
    S = Stream(s)
    s[248:252] = struct.pack("<I", _checksum(bytes(s[256: S.payload])))
    s[252:256] = struct.pack("<I", _checksum(bytes(s[:252])))


def test_reader_rejects_overlapping_units():
    f = _field("normal", (21, 19, 23))
    r = oracle.compress(f, 0.05, [], levels=2, block=4, merge=2)
    s = bytearray(r["stream"])
    S = Stream(s)
    xt = 256 + 16 * S.nblocks * S.nL + 16 * S.nblocks
    # unit 1 starts where unit 0 does: overlapping units, a block left out
    s[xt + 32: xt + 44] = s[xt: xt + 12]
    _resum(s)
    with pytest.raises(oracle.OracleError):
        oracle.stream_info(s)
    # the untouched stream passes the same checks
    t = bytearray(r["stream"])
    _resum(t)
    oracle.stream_info(t)


def test_merge_argument_errors():
    f = _field("normal", (9, 9, 9))
    with pytest.raises(oracle.OracleError):
        oracle.compress(f, 0.05, [0.0], levels=2, block=4, merge=2, error_bound_far=0.5)
    with pytest.raises(oracle.OracleError):
        oracle.compress(f, 0.05, [0.0], levels=2, block=4, merge=17)


def test_extraction_box_over_merged_units():
    """The extraction-side box of a merged stream covers every crossing
    cell: marching cubes over it gives the full field's mesh."""
    f = _field("smooth", (40, 37, 45))
    r = oracle.compress(f, 1e-3, [0.5], levels=3, block=8, merge=3)
    y = oracle.decompress(r["stream"], 0)
    box = oracle.block_box(r["stream"], 0.5, 0.5)
    assert box is not None
    lo, hi = box
    v, t = oracle.mc(y, 0.5)[:2]
    vb, tb = oracle.mc_box(y, lo, hi, 0.5)
    assert len(t) > 0
    assert np.array_equal(v, vb) and np.array_equal(t, tb)
