"""Pins of differentiated error control in the oracle (blocks get different
error bounds, Sec. II.A).

Reading: a block is active when the input on its closed extent crosses a
candidate isovalue (min < k <= max); a point takes the near bound when any
block whose closed extent contains it is active, the far bound otherwise.
The activity and the near set are recomputed here independently (numpy
slices over closed extents), and the consequences the reading implies are
checked: the bounds per point, near points equal to a uniform-bound stream's
values bit for bit, candidate-isovalue meshes identical to the uniform
stream's, no candidates = the far bound everywhere.
"""
import numpy as np
import pytest

import oracle
from paper_2408_05462_amd import inputs


def _nblk(n, B):
    return 1 if n <= 1 else -(-(n - 1) // B)


def _extents(shape, B):
    nb = [_nblk(n, B) for n in shape]
    for bz in range(nb[0]):
        for by in range(nb[1]):
            for bx in range(nb[2]):
                o = (bz * B, by * B, bx * B)
                hi = tuple(min(o[a] + B, shape[a] - 1) for a in range(3))
                yield tuple(slice(o[a], hi[a] + 1) for a in range(3))


def _activity(f, isos, B):
    act = []
    for sl in _extents(f.shape, B):
        mn, mx = float(f[sl].min()), float(f[sl].max())
        act.append(any(mn < k <= mx for k in np.asarray(isos, np.float32).tolist()))
    return np.array(act)


def _near(f, isos, B):
    near = np.zeros(f.shape, bool)
    for a, sl in zip(_activity(f, isos, B), _extents(f.shape, B)):
        if a:
            near[sl] = True
    return near


def _flags(stream):
    I = oracle.stream_info(stream)
    bt = 256 + 16 * I.nblocks * I.levels
    return np.frombuffer(stream[bt: bt + 16 * I.nblocks].tobytes(), np.uint32).reshape(-1, 4)[:, 3]


CASES = [
    # field, shape slice, levels, block, isovalues
    ("grf", (40, 37, 45), 3, 8, [2.0]),
    ("grf", (33, 33, 33), 4, 8, [-2.2, 2.4]),
    ("grf", (17, 30, 9), 3, 4, [1.0]),
    ("smooth", (24, 24, 24), 3, 8, [0.3, 0.7]),
]


def _field(kind, shape):
    if kind == "grf":
        n = max(shape)
        return np.ascontiguousarray(inputs.grf(n, 0.5)[: shape[0], : shape[1], : shape[2]])
    return inputs.gaussians(shape[0], seed=5)


@pytest.mark.parametrize("case", range(len(CASES)))
def test_block_flags_and_per_point_bounds(case):
    kind, shape, nL, B, isos = CASES[case]
    f = _field(kind, shape)
    r = float(f.max() - f.min())
    e, ef = 1e-3 * r, 3e-2 * r
    d = oracle.compress(f, e, isos, levels=nL, block=B, error_bound_far=ef)
    act = _activity(f, isos, B)
    assert 0 < act.sum() < act.size                     # the case exercises both kinds of block
    assert np.array_equal(_flags(d["stream"]), act.astype(np.uint32))
    near = _near(f, isos, B)
    err = np.abs(d["xr"].astype(np.float64) - f)
    assert err[near].max() <= e
    assert err.max() <= ef
    assert err[~near].max() > e                          # the far bound is in use
    y = oracle.decompress(d["stream"])
    assert np.array_equal(y.view(np.uint32), d["xr"].view(np.uint32))
    # near points are the uniform stream's, bit for bit
    u = oracle.compress(f, e, isos, levels=nL, block=B)
    assert np.array_equal(d["xr"][near].view(np.uint32), u["xr"][near].view(np.uint32))
    assert d["stream"].size < u["stream"].size
    assert oracle.stream_verify(d["stream"]) == oracle.OK


@pytest.mark.parametrize("case", range(len(CASES)))
def test_candidate_meshes_equal_the_uniform_streams(case):
    kind, shape, nL, B, isos = CASES[case]
    f = _field(kind, shape)
    r = float(f.max() - f.min())
    y = oracle.decompress(oracle.compress(f, 1e-3 * r, isos, levels=nL, block=B, error_bound_far=5e-2 * r)["stream"])
    yu = oracle.decompress(oracle.compress(f, 1e-3 * r, isos, levels=nL, block=B)["stream"])
    for k in isos:
        assert np.array_equal(oracle.mc_cases(y, k), oracle.mc_cases(f, k))
        v, t, _, _ = oracle.mc(y, k)
        vu, tu, _, _ = oracle.mc(yu, k)
        assert np.array_equal(t, tu)
        assert np.array_equal(v.view(np.uint32), vu.view(np.uint32))


def test_no_candidates_means_the_far_bound_everywhere():
    f = _field("grf", (20, 21, 22))
    d = oracle.compress(f, 0.01, [], levels=3, block=8, error_bound_far=0.2)
    u = oracle.compress(f, 0.2, [], levels=3, block=8)
    assert not _flags(d["stream"]).any()
    assert np.array_equal(d["xr"].view(np.uint32), u["xr"].view(np.uint32))


def test_equal_bounds_give_the_uniform_values():
    f = _field("grf", (20, 21, 22))
    d = oracle.compress(f, 0.05, [0.5], levels=3, block=8, error_bound_far=0.05)
    u = oracle.compress(f, 0.05, [0.5], levels=3, block=8)
    assert np.array_equal(d["xr"].view(np.uint32), u["xr"].view(np.uint32))
    assert oracle.stream_info(d["stream"]).flags & 2
    assert not oracle.stream_info(u["stream"]).flags & 2


def test_lossless_near_blocks():
    f = _field("grf", (24, 24, 24))
    isos = [2.0]
    d = oracle.compress(f, 0.0, isos, levels=3, block=8, error_bound_far=0.1)
    near = _near(f, isos, 8)
    assert near.any() and not near.all()
    assert np.array_equal(d["xr"][near].view(np.uint32), f[near].view(np.uint32))
    assert np.abs(d["xr"] - f).max() <= 0.1
    assert oracle.stream_info(d["stream"]).flags & 7 == 3   # near lossless, differentiated, far lossy


def test_invalid_far_bounds_and_accuracy_requests():
    f = _field("grf", (12, 12, 12))
    for bad in (0.001, float("inf"), float("nan"), -1.0):
        with pytest.raises(oracle.OracleError):
            oracle.compress(f, 0.01, [0.5], levels=2, block=4, error_bound_far=bad)
    s = oracle.compress(f, 0.01, [0.5], levels=2, block=4, error_bound_far=0.1)["stream"]
    # a differentiated stream guarantees its far bound everywhere: requests below it are refused
    assert oracle.decompress_rc(s, 0, 0.05) == oracle.E_ACCURACY
    assert oracle.decompress_rc(s, 0, 0.1) == oracle.OK
