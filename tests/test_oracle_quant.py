"""Pins for the oracle's hierarchy, predictor and quantizer.

Each test checks the oracle against something other than its own code:
closed-form point counts, exact identities of affine/multilinear/quadratic
fields, hand-worked quantizer values and the rounding definition.
"""
import itertools
from fractions import Fraction

import numpy as np
import pytest

import oracle


# ---------------------------------------------------------------- hierarchy

def _count_closed_form(dims, nL):
    """Points per level: m_l = floor((n-1)/2^l)+1 points of the 2^l grid per
    axis; level l holds the 2^l grid minus the 2^(l+1) grid, the top level
    holds the whole 2^(nL-1) grid."""
    def grid(l):
        return int(np.prod([((n - 1) >> l) + 1 for n in dims]))
    L = nL - 1
    return [grid(l) - grid(l + 1) for l in range(L)] + [grid(L)]


@pytest.mark.parametrize("dims,nL", [((9, 10, 17), 3), ((16, 16, 16), 4), ((5, 1, 7), 2), ((33, 20, 12), 5)])
def test_level_counts_closed_form(dims, nL):
    counts = [0] * nL
    for z, y, x in itertools.product(*[range(n) for n in dims]):
        counts[oracle.level_of(x, y, z, nL)] += 1
    assert counts == _count_closed_form(dims, nL)


def test_level_counts_64cubed_three_levels():
    # 64^3 with 3 levels: 16^3 anchors, 32^3-16^3 level-1 points, 64^3-32^3 level-0 points
    assert _count_closed_form((64, 64, 64), 3)[::-1] == [4096, 28672, 229376]


def test_level_examples():
    assert oracle.level_of(0, 0, 0, 4) == 3
    assert oracle.level_of(8, 0, 16, 4) == 3
    assert oracle.level_of(1, 0, 0, 4) == 0
    assert oracle.level_of(2, 4, 6, 4) == 1
    assert oracle.level_of(4, 12, 0, 4) == 2
    assert oracle.level_of(4, 12, 0, 2) == 1   # capped at the top level


# ---------------------------------------------------------------- predictor

def _grid(dims):
    z, y, x = np.meshgrid(*[np.arange(n) for n in dims], indexing="ij")
    return x, y, z


def _clipped(c, h, n):
    return ((c // h) & 1) == 1 and c + h >= n


@pytest.mark.parametrize("nL", [2, 3, 4])
def test_predict_affine_exact(nL):
    """Midpoint averages of an affine field are exact; where the upper parent
    lies outside the domain the lower parent is used, which shifts the
    prediction by -slope*h along that axis."""
    dims = (13, 10, 11)
    sx, sy, sz = 0.5, 0.25, 2.0
    x, y, z = _grid(dims)
    f = (1.0 + sx * x + sy * y + sz * z).astype(np.float32)
    for (zz, yy, xx) in itertools.product(*[range(n) for n in dims]):
        lv = oracle.level_of(xx, yy, zz, nL)
        if lv == nL - 1:
            continue
        h = 1 << lv
        p = oracle.predict(f, xx, yy, zz, lv, nL)
        expect = f[zz, yy, xx]
        expect = expect - sx * h * _clipped(xx, h, dims[2]) - sy * h * _clipped(yy, h, dims[1]) \
            - sz * h * _clipped(zz, h, dims[0])
        assert p == np.float32(expect), (xx, yy, zz, lv)


def test_predict_trilinear_exact():
    """A multilinear field is reproduced exactly at every interior point."""
    dims = (9, 9, 9)
    x, y, z = _grid(dims)
    f = ((x + 1.0) * (y + 2.0) * (z + 3.0)).astype(np.float32)
    nL = 4
    for (zz, yy, xx) in itertools.product(range(9), range(9), range(9)):
        lv = oracle.level_of(xx, yy, zz, nL)
        if lv == nL - 1:
            continue
        assert oracle.predict(f, xx, yy, zz, lv, nL) == f[zz, yy, xx]


def test_predict_quadratic_offset():
    """For f = x^2 the average of (x-h)^2 and (x+h)^2 is x^2 + h^2: pins the
    parent distance h (a stencil at 2h would give 4h^2)."""
    dims = (1, 1, 17)
    f = (np.arange(17, dtype=np.float64) ** 2).astype(np.float32).reshape(dims)
    nL = 4
    for xx in range(17):
        lv = oracle.level_of(xx, 0, 0, nL)
        if lv == nL - 1 or xx + (1 << lv) >= 17:
            continue
        h = 1 << lv
        assert oracle.predict(f, xx, 0, 0, lv, nL) == np.float32(xx * xx + h * h)


def test_predict_uses_reconstructed_parents_only():
    """Changing a non-parent value never changes a prediction."""
    rng = np.random.default_rng(3)
    f = rng.standard_normal((9, 9, 9)).astype(np.float32)
    p0 = oracle.predict(f, 3, 2, 4, 0, 3)   # x odd: parents (2,2,4), (4,2,4) along x only
    g = f.copy()
    g[4, 2, 3] = 100.0                       # the point itself
    g[4, 3, 3] = 100.0                       # a neighbour that is not a parent
    assert oracle.predict(g, 3, 2, 4, 0, 3) == p0
    g[4, 2, 4] = 100.0                       # a parent
    assert oracle.predict(g, 3, 2, 4, 0, 3) != p0


# ---------------------------------------------------------------- quantizer

def test_quantize_worked_example():
    # e = 0.1: inv = fl32(5) = 5, step = fl32(0.2); x - p = 1 -> code 5,
    # 5 * fl32(0.2) = 1.0000000149 rounds to 1.0 in binary32
    q, o, r = oracle.quantize(1.0, 0.0, 0.1)
    assert (q, o, r) == (5, 0, np.float32(1.0))


def test_quantize_round_half_even():
    # e = 0.25: inv = 2, step = 0.5.  d = 0.25 -> 0.5 -> 0 (even); d = 0.75 -> 1.5 -> 2
    assert oracle.quantize(0.25, 0.0, 0.25)[0] == 0
    assert oracle.quantize(0.75, 0.0, 0.25)[0] == 2
    assert oracle.quantize(-0.75, 0.0, 0.25)[0] == -2
    assert oracle.quantize(1.25, 0.0, 0.25)[0] == 2


def test_quantize_bound_and_rounding_property():
    """|q - d/(2e)| <= 1/2 (up to the binary32 rounding of d and 1/(2e)) and
    |x' - x| <= e whenever the value is not an outlier."""
    rng = np.random.default_rng(7)
    for _ in range(3000):
        e = float(10.0 ** rng.uniform(-6, 1))
        p = np.float32(rng.normal(0, 10))
        x = np.float32(p + rng.normal(0, 50 * e))
        q, o, r = oracle.quantize(float(x), float(p), e)
        d = float(np.float32(x - p))
        inv = float(np.float32(1.0 / (2.0 * e)))
        if not o:
            assert abs(q - d * inv) <= 0.5 + 1e-6 * max(1.0, abs(q))
            assert abs(float(r) - float(x)) <= e


def test_quantize_outlier_beyond_qmax():
    q, o, r = oracle.quantize(1000.0, 0.0, 0.001, qmax=32767)  # needs |q| = 500000
    assert (q, o) == (0, 1) and r == np.float32(0.0)
    q, o, r = oracle.quantize(0.01, 0.0, 0.001, qmax=4)        # needs |q| = 5
    assert (q, o) == (0, 1)


def test_quantize_lossless_mode():
    # e = 0: code 0, reconstruction = prediction, outlier unless bitwise equal
    assert oracle.quantize(1.5, 1.5, 0.0) == (0, 0, np.float32(1.5))
    q, o, r = oracle.quantize(1.5, 1.25, 0.0)
    assert (q, o, r) == (0, 1, np.float32(1.25))
    q, o, r = oracle.quantize(-0.0, 0.0, 0.0)   # -0 and +0 differ bitwise
    assert o == 1


def test_rank_counts_not_below():
    iso = [0.5, -1.0, 2.0]
    assert oracle.rank(-2.0, iso) == 0
    assert oracle.rank(-1.0, iso) == 1    # v == k is "not below"
    assert oracle.rank(0.7, iso) == 2
    assert oracle.rank(2.0, iso) == 3


def test_multilinear_closed_form_codes():
    """Multilinear field, dyadic step: anchors code f/step, interior codes 0,
    clipped stencils code (f(c) - f(c'))/step, where c' moves every clipped odd
    axis down by h; every reconstruction is exact."""
    dims = (11, 14, 13)
    nL = 3
    x, y, z = _grid(dims)
    f64 = (x + 1.0) * (y + 3.0) * (2.0 * z + 1.0) / 8.0
    f = f64.astype(np.float32)
    e = 1.0 / 32.0                            # step = 1/16, every value a multiple of 1/8
    r = oracle.compress(f, e, [], levels=nL, block=4)
    assert np.array_equal(r["xr"], f)
    assert not r["flags"].any()

    def fx(cx, cy, cz):
        return Fraction(cx + 1) * (cy + 3) * (2 * cz + 1) / 8

    for (zz, yy, xx) in itertools.product(*[range(n) for n in dims]):
        lv = oracle.level_of(xx, yy, zz, nL)
        if lv == nL - 1:
            expect = fx(xx, yy, zz) * 16
        else:
            h = 1 << lv
            c2 = [xx - h * _clipped(xx, h, dims[2]), yy - h * _clipped(yy, h, dims[1]),
                  zz - h * _clipped(zz, h, dims[0])]
            expect = (fx(xx, yy, zz) - fx(*c2)) * 16
        assert expect.denominator == 1
        assert r["q"][zz, yy, xx] == int(expect), (xx, yy, zz)
