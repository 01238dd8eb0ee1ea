"""Independent pure-Python marching cubes for tiny fields (test helper).

A second derivation of the triangle-table rule and of marching cubes, written
from the rule's statement with different data structures from the C oracle
(corners as coordinate triples, edges as corner pairs, faces as corner sets):

* cell corner (dx,dy,dz) has index dx + 2dy + 4dz and is "below" when f < k;
* an edge is crossed when its two corners differ;
* on a face with two crossed edges they form one segment; on a face with four
  crossed edges, each below corner is cut off by the segment between its two
  edges;
* the segments form disjoint loops; each loop is oriented so that its area
  vector (edge midpoints) points from below to above, started at its smallest
  edge id and fan-triangulated;
* vertices are numbered by (point, axis) in lexicographic point order,
  triangles by (cell, table order); a vertex sits at t = (k-fa)/(fb-fa) along
  its edge, computed in binary32.
"""
from __future__ import annotations

import itertools

import numpy as np

CORNERS = [(dx, dy, dz) for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]  # index = dx+2dy+4dz


def _edges():
    out = []
    for axis in range(3):
        others = [a for a in range(3) if a != axis]
        for r in (0, 1):          # second "other" axis
            for p in (0, 1):      # first "other" axis
                lo = [0, 0, 0]
                lo[others[0]] = p
                lo[others[1]] = r
                hi = list(lo)
                hi[axis] = 1
                out.append((tuple(lo), tuple(hi), axis))
    return out


EDGES = _edges()  # edge id -> (lo corner, hi corner, axis)


def _cidx(c):
    return c[0] + 2 * c[1] + 4 * c[2]


def _faces():
    faces = []
    for axis in range(3):
        for side in (0, 1):
            faces.append([c for c in CORNERS if c[axis] == side])
    return faces


def _edge_of(c0, c1):
    for e, (lo, hi, _) in enumerate(EDGES):
        if {lo, hi} == {c0, c1}:
            return e
    return None


def table():
    """Returns list of 256 lists of (e0, e1, e2) triangles."""
    tab = []
    for case in range(256):
        below = {c: bool((case >> _cidx(c)) & 1) for c in CORNERS}
        adj = {}
        for face in _faces():
            f_edges = [(a, b) for a, b in itertools.combinations(face, 2)
                       if sum(abs(a[i] - b[i]) for i in range(3)) == 1]
            crossed = [_edge_of(a, b) for a, b in f_edges if below[a] != below[b]]
            segs = []
            if len(crossed) == 2:
                segs.append(tuple(crossed))
            elif len(crossed) == 4:
                for c in face:
                    if below[c]:
                        mine = [_edge_of(a, b) for a, b in f_edges if c in (a, b)]
                        segs.append(tuple(mine))
            for a, b in segs:
                adj.setdefault(a, []).append(b)
                adj.setdefault(b, []).append(a)
        assert all(len(v) == 2 for v in adj.values()), case
        seen = set()
        tris = []
        for start in sorted(adj):
            if start in seen:
                continue
            loop = [start]
            seen.add(start)
            prev, cur = start, adj[start][0]
            while cur != start:
                loop.append(cur)
                seen.add(cur)
                nxt = adj[cur][0] if adj[cur][0] != prev else adj[cur][1]
                prev, cur = cur, nxt
            mids = [np.add(EDGES[e][0], EDGES[e][1]) / 2.0 for e in loop]
            area = np.zeros(3)
            for i in range(len(loop)):
                area += np.cross(mids[i], mids[(i + 1) % len(loop)])
            grad = np.zeros(3)
            for e in loop:
                lo, hi, axis = EDGES[e]
                grad[axis] += 1.0 if below[lo] else -1.0
            if float(area @ grad) < 0:
                loop = [loop[0]] + loop[1:][::-1]
            for i in range(1, len(loop) - 1):
                tris.append((loop[0], loop[i], loop[i + 1]))
        tab.append(tris)
    return tab


_TAB = None


def mc(f: np.ndarray, k: float, spacing: float = 1.0):
    """Marching cubes on a tiny [nz][ny][nx] float32 field."""
    global _TAB
    if _TAB is None:
        _TAB = table()
    f = np.asarray(f, np.float32)
    k = np.float32(k)
    nz, ny, nx = f.shape
    vid = {}
    verts = []
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                for axis, (ox, oy, oz) in enumerate(((1, 0, 0), (0, 1, 0), (0, 0, 1))):
                    X, Y, Z = x + ox, y + oy, z + oz
                    if X >= nx or Y >= ny or Z >= nz:
                        continue
                    fa, fb = f[z, y, x], f[Z, Y, X]
                    if (fa < k) == (fb < k):
                        continue
                    t = np.float32(np.float32(k - fa) / np.float32(fb - fa))
                    p = [np.float32(x), np.float32(y), np.float32(z)]
                    p[axis] = np.float32(p[axis] + t)
                    verts.append([np.float32(c * np.float32(spacing)) for c in p])
                    vid[(z, y, x, axis)] = len(verts) - 1
    tris = []
    cases = np.zeros((max(nz - 1, 0), max(ny - 1, 0), max(nx - 1, 0)), np.uint8)
    for z in range(nz - 1):
        for y in range(ny - 1):
            for x in range(nx - 1):
                case = 0
                for c in CORNERS:
                    if f[z + c[2], y + c[1], x + c[0]] < k:
                        case |= 1 << _cidx(c)
                cases[z, y, x] = case
                for tri in _TAB[case]:
                    ids = []
                    for e in tri:
                        lo, hi, axis = EDGES[e]
                        ids.append(vid[(z + lo[2], y + lo[1], x + lo[0], axis)])
                    tris.append(ids)
    return (np.array(verts, np.float32).reshape(-1, 3), np.array(tris, np.int32).reshape(-1, 3), cases)
