"""Pins for the oracle's marching cubes (Sec. I cites marching cubes; Sec. II.B
defines topology preservation through the per-cell case).

The table is generated from a face rule, so it is pinned by structure
(every crossed edge used, loops closed on the cube faces, rotation
invariance), by an independent Python derivation, and by geometry: a sphere's
area and volume converge to 4*pi*r^2 and 4/3*pi*r^3, the mesh is a closed
oriented 2-manifold of Euler characteristic 2, and a tilted plane is
reproduced exactly.
"""
import itertools

import numpy as np
import pytest

import oracle
import ref_mc

CORNERS = [(v & 1, (v >> 1) & 1, (v >> 2) & 1) for v in range(8)]


def _table():
    ntri, tri = oracle.mc_table()
    return [[tuple(t) for t in tri[c][: 3 * ntri[c]].reshape(-1, 3).tolist()] for c in range(256)]


def _edge_corners(e):
    lo, hi, axis = ref_mc.EDGES[e]
    return lo, hi


def test_table_matches_independent_derivation():
    assert _table() == [list(t) for t in ref_mc.table()]


def test_table_structure():
    tab = _table()
    assert tab[0] == [] and tab[255] == []
    for case in range(256):
        below = [(case >> v) & 1 for v in range(8)]
        crossed = set()
        for e in range(12):
            lo, hi = _edge_corners(e)
            if below[lo[0] + 2 * lo[1] + 4 * lo[2]] != below[hi[0] + 2 * hi[1] + 4 * hi[2]]:
                crossed.add(e)
        used = {e for t in tab[case] for e in t}
        assert used == crossed, case
        # boundary of the triangle set: undirected edges used once
        cnt = {}
        for t in tab[case]:
            assert len(set(t)) == 3
            for a, b in ((t[0], t[1]), (t[1], t[2]), (t[2], t[0])):
                key = (min(a, b), max(a, b))
                cnt[key] = cnt.get(key, 0) + 1
        boundary = [k for k, c in cnt.items() if c == 1]
        assert all(c in (1, 2) for c in cnt.values())
        # every boundary segment joins two edges of one cube face and every
        # crossed edge ends exactly two segments (closed loops)
        deg = {}
        for a, b in boundary:
            ca = set(_edge_corners(a))
            cb = set(_edge_corners(b))
            pts = list(ca | cb)
            assert any(all(p[ax] == s for p in pts) for ax in range(3) for s in (0, 1)), (case, a, b)
            deg[a] = deg.get(a, 0) + 1
            deg[b] = deg.get(b, 0) + 1
        assert set(deg) == crossed and all(d == 2 for d in deg.values())


def test_table_small_cases():
    ntri, _ = oracle.mc_table()
    for v in range(8):
        assert ntri[1 << v] == 1          # a single below corner is cut off by one triangle
        assert ntri[255 ^ (1 << v)] == 1  # a single above corner likewise
    assert ntri[0b00001111] == 2          # a whole face below: one quad
    assert ntri[0b00000011] == 2          # two corners along an edge: one quad
    assert ntri[0b01101001] == 4          # checkerboard below corners 0,3,5,6: four corner triangles
    assert ntri[0b10010110] == 4


def _rotations():
    mats = []
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product((1, -1), repeat=3):
            m = np.zeros((3, 3), int)
            for i in range(3):
                m[i, perm[i]] = signs[i]
            if round(np.linalg.det(m)) == 1:
                mats.append(m)
    assert len(mats) == 24
    return mats


def test_triangle_count_rotation_invariant():
    ntri, _ = oracle.mc_table()
    for m in _rotations():
        perm = []
        for c in CORNERS:
            p = m @ (np.array(c) * 2 - 1)
            q = ((p + 1) // 2).astype(int)
            perm.append(int(q[0] + 2 * q[1] + 4 * q[2]))
        for case in range(256):
            rc = 0
            for v in range(8):
                if (case >> v) & 1:
                    rc |= 1 << perm[v]
            assert ntri[rc] == ntri[case]


@pytest.mark.parametrize("seed,shape,k", [(0, (6, 7, 8), 0.1), (1, (9, 5, 4), -0.3), (2, (3, 3, 3), 0.0),
                                          (3, (16, 16, 16), 0.25), (4, (1, 5, 5), 0.0)])
def test_bruteforce_against_python_mc(seed, shape, k):
    f = np.random.default_rng(seed).standard_normal(shape).astype(np.float32)
    if seed == 2:
        f[1, 1, 1] = 0.0          # values equal to k count as "not below"
    v1, t1, c1 = ref_mc.mc(f, k, spacing=2.0)
    v2, t2, counts, rc = oracle.mc(f, k, spacing=2.0)
    assert rc == oracle.OK
    assert np.array_equal(v1.view(np.uint32), v2.view(np.uint32))
    assert np.array_equal(t1, t2)
    if min(shape) > 1:
        assert np.array_equal(c1, oracle.mc_cases(f, k))


def test_capacity_reports_required_sizes():
    f = np.random.default_rng(5).standard_normal((8, 8, 8)).astype(np.float32)
    v, t, counts, rc = oracle.mc(f, 0.0)
    v2, t2, counts2, rc2 = oracle.mc(f, 0.0, cap_v=3, cap_t=2)
    assert rc2 == oracle.E_CAPACITY and counts2 == counts
    assert np.array_equal(v2, v[:3]) and np.array_equal(t2, t[:2])


def _sphere(n, r, c):
    ax = np.arange(n, dtype=np.float64)
    z, y, x = np.meshgrid(ax - c[0], ax - c[1], ax - c[2], indexing="ij")
    return np.sqrt(x * x + y * y + z * z).astype(np.float32), np.float32(r)


def _mesh_stats(v, t):
    a = v[t[:, 0]].astype(np.float64)
    b = v[t[:, 1]].astype(np.float64)
    c = v[t[:, 2]].astype(np.float64)
    cr = np.cross(b - a, c - a)
    area = 0.5 * np.linalg.norm(cr, axis=1).sum()
    vol = np.einsum("ij,ij->i", a, np.cross(b, c)).sum() / 6.0
    return area, vol


@pytest.mark.parametrize("r", [8, 16, 24])
def test_sphere_is_closed_oriented_manifold(r):
    n = 2 * r + 8
    c = (n / 2 - 0.37, n / 2 + 0.21, n / 2 - 0.13)
    f, k = _sphere(n, r, c)
    v, t, counts, rc = oracle.mc(f, k)
    # each undirected edge is used by exactly two triangles, in opposite directions
    directed = {}
    for tri in t:
        for a, b in ((tri[0], tri[1]), (tri[1], tri[2]), (tri[2], tri[0])):
            directed[(a, b)] = directed.get((a, b), 0) + 1
    for (a, b), cnt in directed.items():
        assert cnt == 1 and directed.get((b, a), 0) == 1
    E = len(directed) // 2
    assert len(v) - E + len(t) == 2          # Euler characteristic of a sphere
    area, vol = _mesh_stats(v - np.array([c[2], c[1], c[0]], np.float32), t)
    assert vol > 0                           # normals point outward, toward increasing f
    assert abs(area / (4 * np.pi * r * r) - 1) < 0.12
    assert abs(vol / (4 / 3 * np.pi * r ** 3) - 1) < 0.05


def test_sphere_area_converges():
    errs = []
    for r in (8, 16, 24):
        n = 2 * r + 8
        c = (n / 2 - 0.37, n / 2 + 0.21, n / 2 - 0.13)
        f, k = _sphere(n, r, c)
        v, t, _, _ = oracle.mc(f, k)
        area, vol = _mesh_stats(v, t)
        errs.append((abs(area / (4 * np.pi * r * r) - 1), abs(vol / (4 / 3 * np.pi * r ** 3) - 1)))
    assert errs[0][1] > errs[1][1] > errs[2][1]
    assert errs[2][0] < 0.1 and errs[2][1] < 0.01


def test_tilted_plane_exact():
    """f = x + 2y is linear, so every vertex lies on the plane x + 2y = k and the
    mesh is the exact cross-section of the box: a rectangle of width
    |segment of x + 2y = k in the xy box| and height nz - 1."""
    nz, ny, nx = 6, 9, 14
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    f = (x + 2.0 * y).astype(np.float32)
    k = np.float32(9.5)
    v, t, _, rc = oracle.mc(f, k)
    assert np.max(np.abs(v[:, 0] + 2 * v[:, 1] - k)) < 1e-5
    # segment of x + 2y = 9.5 inside [0,13] x [0,8]: x from 0 to 9.5 (y from 4.75 to 0)
    length = np.hypot(9.5, 4.75)
    area, _ = _mesh_stats(v, t)
    assert area == pytest.approx(length * (nz - 1), rel=1e-5)


def test_spacing_scales_positions():
    f = np.random.default_rng(9).standard_normal((5, 6, 7)).astype(np.float32)
    v1, t1, _, _ = oracle.mc(f, 0.2, spacing=1.0)
    v4, t4, _, _ = oracle.mc(f, 0.2, spacing=4.0)
    assert np.array_equal(t1, t4)
    assert np.array_equal(v4, v1 * np.float32(4.0))
