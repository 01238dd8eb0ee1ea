// mc_table.h -- marching-cubes triangle table, generated at compile time.
//
// Case index: bit v set iff corner v = dx + 2dy + 4dz is below the isovalue.
// Cell edges: 0..3 along x at (dy,dz) = (0,0),(1,0),(0,1),(1,1); 4..7 along y
// at (dx,dz) in the same order; 8..11 along z at (dx,dy).
//
// Rule: on each cube face the crossed edges are joined pairwise -- two
// crossed edges by one segment; four crossed edges (the below corners on a
// diagonal) by the two segments that each isolate one below corner.  Since
// the choice depends only on the face, neighbouring cells agree and the mesh
// is watertight.  Every crossed edge then lies on exactly two segments, so
// the segments form disjoint loops.  A loop is oriented so that its area
// vector (computed on doubled edge-midpoint coordinates, all integers) points
// from the below side to the above side, started at its smallest edge id and
// triangulated as a fan from that edge; loops are taken in order of their
// smallest edge id.
#pragma once

#include <stdint.h>

namespace chr {
namespace mct {

struct Table {
  uint8_t ntri[256];
  int8_t tri[256][15];
};

struct Edge {
  int lo, hi, axis;
};

constexpr Edge edge_of(int e) {
  // returns corner indices of the edge's ends
  int axis = e / 4, i = e % 4;
  int p = i & 1, r = i >> 1;
  int c[3] = {0, 0, 0};
  if (axis == 0) { c[1] = p; c[2] = r; }
  if (axis == 1) { c[0] = p; c[2] = r; }
  if (axis == 2) { c[0] = p; c[1] = r; }
  int lo = c[0] + 2 * c[1] + 4 * c[2];
  c[axis] = 1;
  int hi = c[0] + 2 * c[1] + 4 * c[2];
  return Edge{lo, hi, axis};
}

constexpr int edge_joining(int a, int b) {
  for (int e = 0; e < 12; e++) {
    Edge E = edge_of(e);
    if ((E.lo == a && E.hi == b) || (E.lo == b && E.hi == a)) return e;
  }
  return -1;
}

constexpr Table make_table() {
  Table T{};
  // the 6 faces as cyclic corner sequences: for the face normal to `axis` at
  // `side`, walk the two other axes (p, r): (0,0) (1,0) (1,1) (0,1)
  int face[6][4] = {};
  for (int axis = 0; axis < 3; axis++)
    for (int side = 0; side < 2; side++) {
      int a1 = axis == 0 ? 1 : 0;
      int a2 = axis == 2 ? 1 : 2;
      const int pr[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
      for (int k = 0; k < 4; k++) {
        int c[3] = {0, 0, 0};
        c[axis] = side;
        c[a1] = pr[k][0];
        c[a2] = pr[k][1];
        face[axis * 2 + side][k] = c[0] + 2 * c[1] + 4 * c[2];
      }
    }
  for (int cs = 0; cs < 256; cs++) {
    int link[12][2] = {};
    int nl[12] = {};
    for (int e = 0; e < 12; e++) { link[e][0] = link[e][1] = -1; }
    for (int f = 0; f < 6; f++) {
      int fe[4] = {}, cr[4] = {}, n = 0;
      for (int k = 0; k < 4; k++) {
        int a = face[f][k], b = face[f][(k + 1) % 4];
        fe[k] = edge_joining(a, b);
        cr[k] = ((cs >> a) & 1) != ((cs >> b) & 1);
        n += cr[k];
      }
      if (n == 2) {
        int u = -1, v = -1;
        for (int k = 0; k < 4; k++)
          if (cr[k]) { if (u < 0) u = fe[k]; else v = fe[k]; }
        link[u][nl[u]++] = v;
        link[v][nl[v]++] = u;
      } else if (n == 4) {
        for (int k = 0; k < 4; k++) {
          if (!((cs >> face[f][k]) & 1)) continue;   // isolate each below corner
          int u = fe[(k + 3) % 4], v = fe[k];
          link[u][nl[u]++] = v;
          link[v][nl[v]++] = u;
        }
      }
    }
    bool done[12] = {};
    int nt = 0;
    for (int st = 0; st < 12; st++) {
      if (done[st] || nl[st] == 0) continue;
      int loop[12] = {}, m = 0, prev = -1, cur = st;
      do {
        loop[m++] = cur;
        done[cur] = true;
        int nxt = link[cur][0] != prev ? link[cur][0] : link[cur][1];
        prev = cur;
        cur = nxt;
      } while (cur != st);
      // doubled midpoints, area vector, below->above direction
      long long ax = 0, ay = 0, az = 0, gx = 0, gy = 0, gz = 0;
      for (int i = 0; i < m; i++) {
        Edge A = edge_of(loop[i]), B = edge_of(loop[(i + 1) % m]);
        long long pa[3] = {(A.lo & 1) + (A.hi & 1), ((A.lo >> 1) & 1) + ((A.hi >> 1) & 1),
                           ((A.lo >> 2) & 1) + ((A.hi >> 2) & 1)};
        long long pb[3] = {(B.lo & 1) + (B.hi & 1), ((B.lo >> 1) & 1) + ((B.hi >> 1) & 1),
                           ((B.lo >> 2) & 1) + ((B.hi >> 2) & 1)};
        ax += pa[1] * pb[2] - pa[2] * pb[1];
        ay += pa[2] * pb[0] - pa[0] * pb[2];
        az += pa[0] * pb[1] - pa[1] * pb[0];
        long long sgn = ((cs >> A.lo) & 1) ? 1 : -1;
        if (A.axis == 0) gx += sgn;
        if (A.axis == 1) gy += sgn;
        if (A.axis == 2) gz += sgn;
      }
      if (ax * gx + ay * gy + az * gz < 0) {
        for (int i = 1, j = m - 1; i < j; i++, j--) { int t = loop[i]; loop[i] = loop[j]; loop[j] = t; }
      }
      for (int i = 1; i + 1 < m; i++) {
        T.tri[cs][3 * nt] = (int8_t)loop[0];
        T.tri[cs][3 * nt + 1] = (int8_t)loop[i];
        T.tri[cs][3 * nt + 2] = (int8_t)loop[i + 1];
        nt++;
      }
    }
    T.ntri[cs] = (uint8_t)nt;
    for (int i = 3 * nt; i < 15; i++) T.tri[cs][i] = -1;
  }
  return T;
}

// ---- triangle counts without the table
//
// A loop through k crossed edges is triangulated as a fan of k - 2
// triangles, so a cell with E crossed edges and L loops has E - 2L
// triangles.  On the cube's surface the loops separate the regions around
// the below corners -- joined only along cube edges, since an ambiguous face
// isolates each below corner -- from the regions around the above corners,
// joined along every face they share; a sphere cut by L disjoint loops has
// L + 1 regions.  Hence L > 1 needs two below corners with no path along
// below-below edges or two above corners on no common face.  If no face is
// ambiguous, two below corners sharing a face are joined through that
// face's third or fourth corner, so the below corners can only split as one
// body-diagonal pair with every other corner above; two above corners share
// a face unless they are a body-diagonal pair, and a third above corner
// shares a face with both.  A case that is none of these has one loop and
// E - 2 triangles; the others are corrected from the table.

constexpr int kFaces[6][4] = {{0, 2, 6, 4}, {1, 3, 7, 5}, {0, 1, 5, 4}, {2, 3, 7, 6}, {0, 1, 3, 2}, {4, 5, 7, 6}};
constexpr int kBodyDiag[4][2] = {{0, 7}, {1, 6}, {2, 5}, {3, 4}};

constexpr int crossed_edges(int cs) {
  int n = 0;
  for (int e = 0; e < 12; e++) {
    Edge E = edge_of(e);
    n += ((cs >> E.lo) & 1) != ((cs >> E.hi) & 1);
  }
  return n;
}

// The cases that may hold more than one loop (see above).
constexpr bool multi_loop_possible(int cs) {
  for (int f = 0; f < 6; f++) {
    const int a = (cs >> kFaces[f][0]) & 1, b = (cs >> kFaces[f][1]) & 1;
    const int c = (cs >> kFaces[f][2]) & 1, d = (cs >> kFaces[f][3]) & 1;
    if (a == c && b == d && a != b) return true;   // ambiguous face
  }
  for (int p = 0; p < 4; p++) {
    const int pair = (1 << kBodyDiag[p][0]) | (1 << kBodyDiag[p][1]);
    if (cs == pair || cs == (255 ^ pair)) return true;
  }
  return false;
}

// Triangles of the case minus the single-loop count E - 2 (0 for inactive
// cases and for every case outside multi_loop_possible).
struct LoopFix {
  int8_t d[256];
};

constexpr LoopFix make_loop_fix(const Table &T) {
  LoopFix F{};
  for (int cs = 1; cs < 255; cs++) F.d[cs] = (int8_t)((int)T.ntri[cs] - (crossed_edges(cs) - 2));
  return F;
}

constexpr bool loop_rule_holds(const Table &T) {
  if (T.ntri[0] != 0 || T.ntri[255] != 0) return false;
  for (int cs = 1; cs < 255; cs++)
    if (!multi_loop_possible(cs) && (int)T.ntri[cs] != crossed_edges(cs) - 2) return false;
  return true;
}

}  // namespace mct
}  // namespace chr
