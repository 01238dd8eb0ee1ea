"""Pins for the oracle's compression and reconstruction.

The paper fixes the invariants checked here: the decompressed field keeps
every cell's marching-cubes case (Sec. II.B, definition of topology
preservation) and an error below the vertex-to-isovalue distances keeps the
case (Sec. II.B, edge condition).  The error bound and the lossless round trip
are the defining properties of an error-bounded compressor (Sec. I).
"""
import numpy as np
import pytest

import oracle
from paper_2408_05462_amd import inputs


def cases(f, k):
    return oracle.mc_cases(f, k)


FIELDS = {
    "normal": lambda: np.random.default_rng(11).standard_normal((19, 23, 21)).astype(np.float32),
    "smooth": lambda: inputs.gaussians(24, seed=5),
    "grf": lambda: inputs.grf(24, 0.3),
}


@pytest.mark.parametrize("name", sorted(FIELDS))
@pytest.mark.parametrize("nL,block", [(1, 4), (3, 4), (3, 8), (4, 16), (5, 64)])
def test_error_bound_and_case_identity(name, nL, block):
    f = FIELDS[name]()
    rng = np.random.default_rng(nL * 100 + block)
    isos = list(np.quantile(f, rng.uniform(0.1, 0.9, size=3)).astype(np.float32))
    e = inputs.abs_error_bound(3e-2, f)
    r = oracle.compress(f, e, isos, levels=nL, block=block)
    xr = r["xr"]
    # error bound at every vertex, in double
    assert np.max(np.abs(xr.astype(np.float64) - f.astype(np.float64))) <= e
    # identical case at every cell, for every candidate isovalue, at every level
    for k in isos:
        for l in range(nL):
            s = slice(None, None, 1 << l)
            a, b = f[s, s, s], xr[s, s, s]
            if min(a.shape) > 1:
                assert np.array_equal(cases(a, k), cases(b, k)), (k, l)
    # points stored exactly are exact; codes are zero there
    ex = r["flags"] != 0
    assert np.array_equal(xr[ex].view(np.uint32), f[ex].view(np.uint32))
    assert not r["q"][ex].any()


def test_correction_needed_without_it():
    """The chosen bound is loose enough that quantization alone would change
    cases: corrections do occur, so the identity above is not vacuous."""
    f = FIELDS["normal"]()
    isos = [0.0, 0.5]
    r = oracle.compress(f, inputs.abs_error_bound(3e-2, f), isos, levels=3, block=8)
    assert (r["flags"] & 2).sum() > 0


@pytest.mark.parametrize("nL", [1, 2, 4])
def test_lossless_at_zero_error(nL):
    f = np.random.default_rng(2).standard_normal((9, 12, 17)).astype(np.float32)
    f[0, 0, 0] = -0.0
    f[1, 1, 1] = 0.0
    r = oracle.compress(f, 0.0, [0.1], levels=nL, block=8)
    assert np.array_equal(r["xr"].view(np.uint32), f.view(np.uint32))
    y = oracle.decompress(r["stream"])
    assert np.array_equal(y.view(np.uint32), f.view(np.uint32))


def test_no_corrections_when_every_vertex_is_far_from_every_isovalue():
    """Sec. II.B: an error smaller than the distance to k keeps the side."""
    f = FIELDS["smooth"]()
    isos = np.array([0.2, 0.45], np.float32)
    dist = np.min(np.abs(f[..., None].astype(np.float64) - isos.astype(np.float64)), axis=-1).min()
    r = oracle.compress(f, 0.99 * dist, isos, levels=3, block=8)
    assert not (r["flags"] & 2).any()


@pytest.mark.parametrize("c,expect_corr", [(1.1, True), (1.0, False), (0.5, True), (0.9, False)])
def test_constant_field_equal_to_isovalue(c, expect_corr):
    """Constant field c equal to the isovalue k.  An anchor codes
    q = rint(c/(2e)) and reconstructs q*step; the vertex drops below k exactly
    when q*step < c, and is then corrected.  Every finer point predicts the
    anchors' common value and codes 0."""
    e = 0.03
    f = np.full((9, 9, 9), c, np.float32)
    r = oracle.compress(f, e, [c], levels=3, block=8)
    step = np.float32(2 * e)
    qa = np.rint(np.float32(np.float32(c) * np.float32(1 / (2 * e))))
    anchor_val = np.float32(np.float32(qa) * step)
    assert (anchor_val < np.float32(c)) == expect_corr
    anchors = np.zeros(f.shape, bool)
    anchors[::4, ::4, ::4] = True
    corr = (r["flags"] & 2) != 0
    if expect_corr:
        assert np.array_equal(corr, anchors)
        assert np.all(r["xr"] == np.float32(c))
    else:
        assert not corr.any()
        assert np.all(r["q"][anchors] == qa)
    assert not r["q"][~anchors].any()


def test_paper_error_translation_and_the_vertex_gap():
    """Sec. II.B three-step procedure: with e < min(D) no vertex on a crossing
    edge changes side.  A vertex on no crossing edge can still be closer to k
    than min(D) and flip; the per-vertex check corrects it, and every case
    survives.  (Seeded construction: two half-spaces on either side of k plus
    one vertex 0.01 above k inside the upper half-space.)"""
    n = 12
    rng = np.random.default_rng(1)
    f = rng.uniform(1.0, 3.0, size=(n, n, n)).astype(np.float32)
    f[:, :, : n // 2] *= -1
    k = np.float32(rng.uniform(-0.5, 0.5))
    gap = (6, 6, int(rng.integers(7, 11)))
    f[gap] = np.float32(k + 0.01)
    dmin, nd = oracle.topology_error_bound(f, [k])
    assert 0 < dmin < np.inf and nd > 0
    e = 0.99 * dmin
    r = oracle.compress(f, e, [k], levels=2, block=4)
    corr = (r["flags"] & 2) != 0
    assert corr[gap]                   # the gap vertex had to be corrected
    # no corrected vertex lies on a crossing edge of the original field
    below = f < k
    on_cross = np.zeros_like(below)
    for a in range(3):
        d = np.diff(below.astype(np.int8), axis=a) != 0
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[a] = slice(0, -1)
        sl_hi[a] = slice(1, None)
        on_cross[tuple(sl_lo)] |= d
        on_cross[tuple(sl_hi)] |= d
    assert not on_cross[gap]
    assert not (corr & on_cross).any()
    assert np.array_equal(cases(f, k), cases(r["xr"], k))


def test_topology_bound_nth_smallest():
    f = np.array([[[0.0, 1.0, 3.0, 10.0]]], np.float32)
    # k = 2: one crossing edge (1, 3) -> D = {1, 1}; k = 5: edge (3, 10) -> D = {2, 5}
    r1, n1 = oracle.topology_error_bound(f, [2.0, 5.0], nth=1)
    r3, _ = oracle.topology_error_bound(f, [2.0, 5.0], nth=3)
    r4, _ = oracle.topology_error_bound(f, [2.0, 5.0], nth=4)
    assert (r1, n1, r3, r4) == (1.0, 4, 2.0, 5.0)


@pytest.mark.parametrize("block", [4, 8, 12, 64])
def test_blocks_change_bytes_not_values(block):
    """Closed blocks: every stencil of a block's point lies inside the block,
    so codes and reconstructions do not depend on the block size."""
    f = FIELDS["grf"]()
    e = inputs.abs_error_bound(1e-2, f)
    ref = oracle.compress(f, e, [0.1], levels=3, block=4)
    r = oracle.compress(f, e, [0.1], levels=3, block=block)
    assert np.array_equal(r["q"], ref["q"])
    assert np.array_equal(r["flags"], ref["flags"])
    assert np.array_equal(r["xr"].view(np.uint32), ref["xr"].view(np.uint32))


@pytest.mark.parametrize("nL,block", [(3, 4), (4, 8), (2, 64)])
def test_reconstruct_every_level(nL, block):
    f = FIELDS["normal"]()
    r = oracle.compress(f, 0.05, [0.2], levels=nL, block=block)
    for l in range(nL):
        s = slice(None, None, 1 << l)
        y = oracle.decompress(r["stream"], l)
        assert np.array_equal(y.view(np.uint32), r["xr"][s, s, s].view(np.uint32))


def test_stream_codes_and_header():
    f = FIELDS["normal"]()
    e = 0.02
    r = oracle.compress(f, e, [0.5, -0.25, 0.5], levels=3, block=8)
    q, ex = oracle.stream_codes(r["stream"])
    assert np.array_equal(q, r["q"])
    assert np.array_equal(ex, (r["flags"] != 0).astype(np.uint8))
    info = oracle.stream_info(r["stream"])
    assert tuple(info.dims) == f.shape
    assert info.n_iso == 2 and list(info.iso)[:2] == [-0.25, 0.5]   # sorted, de-duplicated
    assert info.vmin == f.min() and info.vmax == f.max()
    assert info.n_outlier == int((r["flags"] & 1).sum())
    assert info.n_corrected == int((r["flags"] >> 1).sum())
    assert info.total_bytes == len(r["stream"])
    assert info.error_bound == e


def test_block_index_is_min_max_of_closed_block():
    f = FIELDS["grf"]()
    B = 8
    r = oracle.compress(f, 0.01, [0.0], levels=3, block=B)
    mins, maxs = oracle.block_index(r["stream"])
    nb = [max(1, -(-(n - 1) // B)) for n in f.shape]
    b = 0
    for bz in range(nb[0]):
        for by in range(nb[1]):
            for bx in range(nb[2]):
                sl = tuple(slice(i * B, i * B + B + 1) for i in (bz, by, bx))
                blk = r["xr"][sl]
                assert mins[b] == blk.min() and maxs[b] == blk.max()
                b += 1


def test_corruption_is_detected():
    f = FIELDS["normal"]()
    r = oracle.compress(f, 0.05, [0.0], levels=3, block=8)
    s = r["stream"]
    assert oracle.stream_verify(s) == oracle.OK
    rng = np.random.default_rng(0)
    for pos in list(rng.integers(0, len(s), 40)) + [0, 100, 252, 300, len(s) - 1]:
        t = s.copy()
        t[pos] ^= 0x10
        assert oracle.stream_verify(t) == oracle.E_CORRUPT, pos
    assert oracle.stream_verify(s[: len(s) - 8]) == oracle.E_CORRUPT


def test_error_statuses():
    f = FIELDS["normal"]()
    r = oracle.compress(f, 0.05, [0.0], levels=3, block=8)
    assert oracle.decompress_rc(r["stream"], 0, 0.01) == oracle.E_ACCURACY
    assert oracle.decompress_rc(r["stream"], 3, 0.05) == oracle.E_LEVEL
    g = f.copy()
    g[1, 2, 3] = np.nan
    with pytest.raises(oracle.OracleError) as ei:
        oracle.compress(g, 0.05, [0.0], levels=3, block=8)
    assert ei.value.rc == oracle.E_INVAL
    with pytest.raises(oracle.OracleError):
        oracle.compress(f, 0.05, [0.0], levels=3, block=6)   # block not a multiple of 4
