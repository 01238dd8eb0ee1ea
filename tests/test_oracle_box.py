"""Pins of block merging for extraction (the blocks that can hold an
isosurface merged into one rectangular grid, Sec. II.A).

The merged box is recomputed here from the reconstruction's per-block
ranges (numpy, closed extents); marching cubes over the box must give the
full field's mesh bit for bit (every crossing cell lies in a merged block,
and lexicographic order restricted to a box keeps the relative order of
points and cells).
"""
import numpy as np
import pytest

import oracle
from paper_2408_05462_amd import inputs


def _nblk(n, B):
    return 1 if n <= 1 else -(-(n - 1) // B)


def _box_here(y, B, kmin, kmax):
    lo, hi, found = [10 ** 9] * 3, [-1] * 3, False
    nb = [_nblk(n, B) for n in y.shape]
    for bz in range(nb[0]):
        for by in range(nb[1]):
            for bx in range(nb[2]):
                o = (bz * B, by * B, bx * B)
                h = tuple(min(o[a] + B, y.shape[a] - 1) for a in range(3))
                v = y[o[0]: h[0] + 1, o[1]: h[1] + 1, o[2]: h[2] + 1]
                mn, mx = float(v.min()), float(v.max())
                if mn < mx and mn < kmax and kmin <= mx:
                    found = True
                    lo = [min(lo[a], o[a]) for a in range(3)]
                    hi = [max(hi[a], h[a]) for a in range(3)]
    return (tuple(lo), tuple(hi)) if found else None


def _blobs(shape):
    # two separated Gaussian blobs: isosurfaces near their peaks are local
    z, y, x = np.meshgrid(*[np.arange(n, dtype=np.float64) for n in shape], indexing="ij")
    f = np.exp(-((z - 8) ** 2 + (y - 9) ** 2 + (x - 10) ** 2) / 18.0)
    f += 0.8 * np.exp(-((z - 28) ** 2 + (y - 30) ** 2 + (x - 33) ** 2) / 12.0)
    return f.astype(np.float32)


CASES = [
    ("blobs", (40, 41, 45), 3, 8, [0.5, 0.9]),
    ("grf", (33, 35, 31), 3, 4, [1.8]),
    ("grf", (24, 24, 24), 4, 8, [0.0]),
]


def _field(kind, shape):
    if kind == "blobs":
        return _blobs(shape)
    n = max(shape)
    return np.ascontiguousarray(inputs.grf(n, 0.4)[: shape[0], : shape[1], : shape[2]])


@pytest.mark.parametrize("case", range(len(CASES)))
def test_box_recomputed_and_meshes_identical(case):
    kind, shape, nL, B, isos = CASES[case]
    f = _field(kind, shape)
    r = float(f.max() - f.min())
    d = oracle.compress(f, 1e-3 * r, isos, levels=nL, block=B)
    y = oracle.decompress(d["stream"])
    for k in isos:
        box = oracle.block_box(d["stream"], k, k)
        assert box == _box_here(y, B, np.float32(k), np.float32(k))
        v, t, _, _ = oracle.mc(y, k)
        vb, tb = oracle.mc_box(y, box[0], box[1], k)
        assert np.array_equal(tb, t)
        assert np.array_equal(vb.view(np.uint32), v.view(np.uint32))
    # a range: the union of the boxes of its isovalues
    box = oracle.block_box(d["stream"], min(isos), max(isos))
    assert box == _box_here(y, B, np.float32(min(isos)), np.float32(max(isos)))


def test_local_isosurface_gives_a_small_box():
    f = _blobs((40, 41, 45))
    d = oracle.compress(f, 1e-4, [0.9], levels=3, block=8)
    lo, hi = oracle.block_box(d["stream"], 0.9, 0.9)
    vol = np.prod([h - l + 1 for l, h in zip(lo, hi)])
    assert vol < 0.1 * f.size                             # only the first blob's neighbourhood
    y = oracle.decompress(d["stream"])
    v, t, _, _ = oracle.mc(y, 0.9)
    assert t.shape[0] > 0
    # a box that misses part of the surface loses triangles
    vb, tb = oracle.mc_box(y, lo, ((lo[0] + hi[0]) // 2, hi[1], hi[2]), 0.9)
    assert tb.shape[0] < t.shape[0]


def test_no_box_outside_the_range_and_bad_boxes():
    f = _blobs((20, 21, 22))
    d = oracle.compress(f, 1e-4, [0.5], levels=2, block=4)
    assert oracle.block_box(d["stream"], 5.0, 6.0) is None
    with pytest.raises(oracle.OracleError):
        oracle.mc_box(f, (0, 0, 0), (20, 5, 5), 0.5)      # beyond the field
    with pytest.raises(oracle.OracleError):
        oracle.mc_box(f, (5, 0, 0), (4, 5, 5), 0.5)       # lo > hi
