// Lattice layout of the fine mesh for the mass-matrix solves.
//
// The fine mesh is k uniform 4:1 refinements of the coarse mesh, so inside a
// coarse triangle T = (v0, v1, v2) the fine nodes are the points of a
// triangular lattice with m = 2^k steps per edge: (n0 v0 + a v1 + b v2) / m,
// n0 = m - a - b (the integer barycentric coordinates of the prolongation
// code).  Every fine triangle inside T is a translate or a point reflection
// of T scaled by 1/m, so it has area |T| / 4^k, and its edges are parallel to
// T's.  The P1 mass matrix therefore needs neither stored values nor column
// indices away from the coarse vertices:
//   node interior to T (a, b >= 1, a + b <= m - 1): the six neighbours
//     (a+-1, b), (a, b+-1), (a+1, b-1), (a-1, b+1); every edge is shared by
//     two fine triangles of T: M_ij = 2 A / 12, M_ii = 6 A / 6 (A = |T|/4^k);
//   node inside a coarse edge between T1 and T2 (fine areas A1, A2; A2 = 0 on
//     the boundary): two neighbours along the edge with M = (A1 + A2) / 12,
//     two neighbours inside each T_j with M = 2 A_j / 12, M_ii = (A1 + A2)/2;
//   coarse vertex: any valence; its row of the assembled matrix, kept as a
//     fixed-width table with lattice column indices (the diagonal first).
// Vectors in this layout hold, in order: the interior nodes of every coarse
// triangle (triangle-major; see lat_islot for the order within a triangle),
// the m - 1 inner nodes of every coarse edge (from its lower-numbered end),
// the coarse vertices.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#if defined(__HIPCC__)
#define CGP_HD __host__ __device__
#else
#define CGP_HD
#endif

namespace cgp {

struct LatEdgeRec;

struct LatDev {
  int32_t m;      // 2^levels
  int32_t nI;     // interior nodes per coarse triangle, (m-1)(m-2)/2
  int32_t nT, nE, nV;
  int32_t EB, VB; // first edge node, first vertex node
  const int32_t* tri_v;   // [3 nT] coarse triangle vertices
  const int32_t* tri_e;   // [3 nT] (edge << 1) | reversed, local edge j = v_j -> v_{j+1}
  const int32_t* edge_v;  // [2 nE] lower, higher vertex
  const int32_t* edge_t;  // [2 nE] (T << 2) | j of the one or two triangles, -1 if none
  const double* af;       // [nT] fine triangle area |T| / 4^k
  const uint8_t* ldir;    // [N] velocity-Dirichlet flag per lattice node
  const int32_t* lat_of;  // [N] mesh node -> lattice node
  // rows of the coarse vertices of the assembled mass matrix, column major
  // [vw][nV]: entry k of vertex v at [k * nV + v]; slot 0 the diagonal, then
  // the other entries in CSR order; short rows padded with (VB + v, 0)
  int32_t vw;
  const int32_t* vcol;    // lattice column indices
  const double* vval;     // values
  const LatEdgeRec* erec; // [nE] per coarse edge (Lat<M>::edge_record), or nullptr
};

// Per coarse edge, what the rows of its inner nodes read besides their own
// values, so that a row costs one record load instead of the edge's triangle
// and table lookups: for each adjacent triangle q, the lattice indices of the
// row of points one step inside it, parallel to the edge (pts[q][y], y = 0 ..
// m - 1: point (y, 1), (m - 1 - y, y) or (1, y) of the triangle for the
// edge as its local edge 0, 1 or 2; the node at t steps from the edge's lower
// end neighbours points p and p - 1 of that row, p = t, or m - t when the
// row runs the other way) and the triangle's fine area; the edge's two
// vertices.
constexpr int kLatMaxM = 8;
struct LatEdgeRec {
  int32_t pts[2][kLatMaxM];
  double A[2];
  int32_t v[2];     // lower, higher vertex (coarse numbering)
  int32_t meta[2];  // bit 0: triangle q present; bit 1: p = m - t
};
static_assert(sizeof(LatEdgeRec) == 96, "edge record");

// first lattice index of interior row a (1 <= a <= m-2) within a triangle
CGP_HD constexpr int32_t lat_rowoff(int32_t m, int32_t a) {
  return (a - 1) * (m - 1) - ((a - 1) * a) / 2;
}

// position of the interior point (a, b) (a, b >= 1, a + b <= m - 1) in its
// triangle's interior range.  m <= 4: rows a = 1 .. m-2 of b = 1 .. m-1-a.
// m = 8: first the 15 points next to the edges, as one ring -- edge 0's
// first row (b = 1, a = 1..6), edge 1's (a + b = 7, b = 2..6), edge 2's
// (a = 1, b = 5..2) -- then the 6 inner points by rows, so that the values an
// edge node's stencil reads inside a triangle (that triangle's first row
// along the edge) lie in one run of 6 consecutive nodes (for edge 2, two
// runs: positions 10..14 and 0).
CGP_HD constexpr int32_t lat_islot(int32_t m, int32_t a, int32_t b) {
  if (m != 8) return lat_rowoff(m, a) + (b - 1);
  if (b == 1) return a - 1;
  if (a + b == 7) return 4 + b;
  if (a == 1) return 16 - b;
  return 15 + (a - 2) * 3 - ((a - 2) * (a - 3)) / 2 + (b - 2);
}

// lattice index of point (a, b) of coarse triangle T (0 <= a, b; a + b <= m)
CGP_HD inline int32_t lat_index(const LatDev& L, int32_t T, int32_t a, int32_t b) {
  const int32_t m = L.m;
  if (a >= 1 && b >= 1 && a + b <= m - 1) return T * L.nI + lat_islot(m, a, b);
  if (a == 0 && b == 0) return L.VB + L.tri_v[3 * T];
  if (b == 0 && a == m) return L.VB + L.tri_v[3 * T + 1];
  if (a == 0 && b == m) return L.VB + L.tri_v[3 * T + 2];
  int32_t j, p;  // local edge and steps from its first vertex
  if (b == 0) {
    j = 0;
    p = a;
  } else if (a + b == m) {
    j = 1;
    p = b;
  } else {
    j = 2;
    p = m - b;
  }
  const int32_t e = L.tri_e[3 * T + j];
  const int32_t t = (e & 1) ? m - p : p;
  return L.EB + (e >> 1) * (m - 1) + (t - 1);
}

// Index arithmetic with the lattice size m = M fixed at compile time (M in
// {1, 2, 4, 8}): constant divisions, an unrolled row decode, and stencil
// indices computed from a triangle's edge codes and vertices held in
// registers (LatTri), so that a node's neighbours cost no dependent loads.
struct LatTri {
  int32_t te[3], tv[3];
};

template <int M>
struct Lat {
  static constexpr int32_t kM = M;
  static constexpr int32_t NI = (M - 1) * (M - 2) / 2;  // interior nodes per triangle

  CGP_HD static LatTri tri(const LatDev& L, int32_t T) {
    LatTri t;
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      t.te[j] = L.tri_e[3 * T + j];
      t.tv[j] = L.tri_v[3 * T + j];
    }
    return t;
  }

  // node of local edge code e at p steps from the edge's first vertex v_j
  CGP_HD static int32_t edge_pt(const LatDev& L, int32_t e, int32_t p) {
    const int32_t t = (e & 1) ? M - p : p;
    return L.EB + (e >> 1) * (M - 1) + (t - 1);
  }

  // lattice index of point (a, b) of T (0 <= a, b; a + b <= M)
  CGP_HD static int32_t index(const LatDev& L, int32_t T, const LatTri& t, int32_t a, int32_t b) {
    if (a >= 1 && b >= 1 && a + b <= M - 1) return T * NI + lat_islot(M, a, b);
    if (b == 0) return a == 0 ? L.VB + t.tv[0] : (a == M ? L.VB + t.tv[1] : edge_pt(L, t.te[0], a));
    if (a + b == M) return b == M ? L.VB + t.tv[2] : edge_pt(L, t.te[1], b);
    return edge_pt(L, t.te[2], M - b);  // a == 0, 0 < b < M
  }

  // the seven-point stencil of the interior node l = (a, b) of T: nb[0] = l,
  // then (a+1, b), (a, b+1), (a-1, b), (a, b-1), (a+1, b-1), (a-1, b+1).
  // Each neighbour is interior (a fixed offset in the row layout) or one
  // known point of an edge of T, never a vertex: one select each.
  CGP_HD static void interior_nbrs(const LatDev& L, int32_t l, int32_t a, int32_t b,
                                   const LatTri& t, int32_t (&nb)[7]) {
    if constexpr (M == 8) {  // ring order: each neighbour from its point
      const int32_t T = l / NI;
      nb[0] = l;
      nb[1] = index(L, T, t, a + 1, b);
      nb[2] = index(L, T, t, a, b + 1);
      nb[3] = index(L, T, t, a - 1, b);
      nb[4] = index(L, T, t, a, b - 1);
      nb[5] = index(L, T, t, a + 1, b - 1);
      nb[6] = index(L, T, t, a - 1, b + 1);
      return;
    }
    const int32_t up = M - 1 - a, dn = M - a;  // row offsets to rows a + 1 and a - 1
    const bool in_hi = a + b + 1 <= M - 1;
    nb[0] = l;
    nb[1] = in_hi ? l + up : edge_pt(L, t.te[1], b);
    nb[2] = in_hi ? l + 1 : edge_pt(L, t.te[1], b + 1);
    nb[3] = a >= 2 ? l - dn : edge_pt(L, t.te[2], M - b);
    nb[4] = b >= 2 ? l - 1 : edge_pt(L, t.te[0], a);
    nb[5] = b >= 2 ? l + up - 1 : edge_pt(L, t.te[0], a + 1);
    nb[6] = a >= 2 ? l - dn + 1 : edge_pt(L, t.te[2], M - b - 1);
  }

  // triangle and point of an interior node l < EB
  CGP_HD static void interior(int32_t l, int32_t& T, int32_t& a, int32_t& b) {
    constexpr int32_t D = NI > 0 ? NI : 1;
    T = l / D;
    int32_t r = l - T * D;
    if constexpr (M == 8) {  // inverse of lat_islot
      if (r < 6) {
        a = r + 1;
        b = 1;
      } else if (r < 11) {
        b = r - 4;
        a = 7 - b;
      } else if (r < 15) {
        a = 1;
        b = 16 - r;
      } else if (r < 18) {
        a = 2;
        b = r - 13;
      } else if (r < 20) {
        a = 3;
        b = r - 16;
      } else {
        a = 4;
        b = 2;
      }
      return;
    }
    a = 1;
#pragma unroll
    for (int32_t k = 1; k <= M - 3; ++k) {
      const int32_t len = M - 1 - k;  // length of row k
      const bool next = a == k && r >= len;
      r = next ? r - len : r;
      a = next ? k + 1 : a;
    }
    b = r + 1;
  }

  // coarse edge and steps from its lower end of an edge node EB <= l < VB
  CGP_HD static void edge(const LatDev& L, int32_t l, int32_t& E, int32_t& t) {
    constexpr int32_t D = M > 1 ? M - 1 : 1;
    E = (l - L.EB) / D;
    t = (l - L.EB) - E * D + 1;
  }

  // point (a, b) in T of the node at t steps from the lower end of T's local
  // edge j
  CGP_HD static void edge_point(const LatTri& tr, int32_t j, int32_t t, int32_t& a, int32_t& b) {
    const int32_t e = j == 0 ? tr.te[0] : (j == 1 ? tr.te[1] : tr.te[2]);
    const int32_t p = (e & 1) ? M - t : t;  // steps from v_j
    a = j == 0 ? p : (j == 1 ? M - p : 0);
    b = j == 0 ? 0 : (j == 1 ? p : M - p);
  }

  // the record of coarse edge E (set-up; see LatEdgeRec).  The point at
  // steps s from v_j is (s, 0), (m - s, s) or (0, m - s) on local edge 0, 1
  // or 2, and its two inner neighbours are points s and s - 1 (edges 0, 1) or
  // m - s and m - s - 1 (edge 2) of the inner row.
  static LatEdgeRec edge_record(const LatDev& L, int32_t E) {
    static_assert(M <= kLatMaxM, "edge record size");
    LatEdgeRec r{};
    r.v[0] = L.edge_v[2 * E];
    r.v[1] = L.edge_v[2 * E + 1];
    for (int q = 0; q < 2; ++q) {
      const int32_t tj = L.edge_t[2 * E + q];
      if (tj < 0) continue;
      const int32_t T = tj >> 2, j = tj & 3;
      const LatTri tr = tri(L, T);
      const bool rev = ((tr.te[j] & 1) != 0) != (j == 2);
      r.meta[q] = 1 | (rev ? 2 : 0);
      for (int32_t y = 0; y < M; ++y) {
        const int32_t a = j == 0 ? y : (j == 1 ? M - 1 - y : 1);
        const int32_t b = j == 0 ? 1 : y;
        r.pts[q][y] = index(L, T, tr, a, b);
      }
      r.A[q] = L.af[T];
    }
    return r;
  }
};

// (M x)_l for NR interleaved components (x(idx, d) reads component d of
// lattice node idx) and the diagonal M_ll
template <int NR, int M, class X>
CGP_HD inline void lat_apply(const LatDev& L, int32_t l, X x, double (&y)[NR], double& diag) {
  using G = Lat<M>;
  if (l < L.EB) {
    int32_t T, a, b;
    G::interior(l, T, a, b);
    const LatTri t = G::tri(L, T);
    int32_t st[7];
    G::interior_nbrs(L, l, a, b, t, st);
    const int32_t nb[6] = {st[4], st[2], st[1], st[5], st[3], st[6]};
    const double A = L.af[T];
    diag = A;
#pragma unroll
    for (int d = 0; d < NR; ++d) {
      const double s = ((x(nb[0], d) + x(nb[1], d)) + (x(nb[2], d) + x(nb[3], d))) +
                       (x(nb[4], d) + x(nb[5], d));
      y[d] = A * x(l, d) + (A / 6.0) * s;
    }
    return;
  }
  if (l < L.VB) {
    int32_t E, t;
    G::edge(L, l, E, t);
    double acc[NR];
    double asum = 0.0;
#pragma unroll
    for (int d = 0; d < NR; ++d) acc[d] = 0.0;
    if (L.erec) {  // the same reads and operations, from the edge's record
      const LatEdgeRec& R = L.erec[E];
      const int32_t prev = t == 1 ? L.VB + R.v[0] : l - 1;
      const int32_t next = t == M - 1 ? L.VB + R.v[1] : l + 1;
      for (int q = 0; q < 2; ++q) {
        const int32_t meta = R.meta[q];
        if (!(meta & 1)) continue;
        const int32_t p = (meta & 2) ? M - t : t;
        const int32_t i1 = R.pts[q][p], i2 = R.pts[q][p - 1];
        const double A = R.A[q];
        asum += A;
#pragma unroll
        for (int d = 0; d < NR; ++d) acc[d] += (A / 6.0) * (x(i1, d) + x(i2, d));
      }
      diag = 0.5 * asum;
#pragma unroll
      for (int d = 0; d < NR; ++d)
        y[d] = diag * x(l, d) + (asum / 12.0) * (x(prev, d) + x(next, d)) + acc[d];
      return;
    }
    const int32_t prev = t == 1 ? L.VB + L.edge_v[2 * E] : l - 1;
    const int32_t next = t == M - 1 ? L.VB + L.edge_v[2 * E + 1] : l + 1;
    for (int q = 0; q < 2; ++q) {
      const int32_t tj = L.edge_t[2 * E + q];
      if (tj < 0) continue;
      const int32_t T = tj >> 2, j = tj & 3;
      const LatTri tr = G::tri(L, T);
      int32_t a, b;
      G::edge_point(tr, j, t, a, b);
      // the two neighbours inside T, one step off the edge towards its interior
      int32_t i1, i2;
      if (j == 0) {
        i1 = G::index(L, T, tr, a, 1);
        i2 = G::index(L, T, tr, a - 1, 1);
      } else if (j == 1) {
        i1 = G::index(L, T, tr, a - 1, b);
        i2 = G::index(L, T, tr, a, b - 1);
      } else {
        i1 = G::index(L, T, tr, 1, b);
        i2 = G::index(L, T, tr, 1, b - 1);
      }
      const double A = L.af[T];
      asum += A;
#pragma unroll
      for (int d = 0; d < NR; ++d) acc[d] += (A / 6.0) * (x(i1, d) + x(i2, d));
    }
    diag = 0.5 * asum;
#pragma unroll
    for (int d = 0; d < NR; ++d)
      y[d] = diag * x(l, d) + (asum / 12.0) * (x(prev, d) + x(next, d)) + acc[d];
    return;
  }
  // coarse vertex: its table row, four entries' loads issued at a time
  const int32_t v = l - L.VB, nV = L.nV;
  diag = L.vval[v];
#pragma unroll
  for (int d = 0; d < NR; ++d) y[d] = 0.0;
  for (int32_t k0 = 0; k0 < L.vw; k0 += 4) {
    int32_t lc[4];
    double mv[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const bool in = k0 + q < L.vw;
      lc[q] = in ? L.vcol[(int64_t)(k0 + q) * nV + v] : l;
      mv[q] = in ? L.vval[(int64_t)(k0 + q) * nV + v] : 0.0;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      if (k0 + q >= L.vw) break;
#pragma unroll
      for (int d = 0; d < NR; ++d) y[d] += mv[q] * x(lc[q], d);
    }
  }
}

// M_ll alone
CGP_HD inline double lat_diag(const LatDev& L, int32_t l) {
  if (l < L.EB) return L.af[l / L.nI];
  if (l < L.VB) {
    const int32_t E = (l - L.EB) / (L.m - 1);
    double asum = 0.0;
    for (int q = 0; q < 2; ++q) {
      const int32_t tj = L.edge_t[2 * E + q];
      if (tj >= 0) asum += L.af[tj >> 2];
    }
    return 0.5 * asum;
  }
  return L.vval[l - L.VB];
}

// calls f(Lat<M>{}) for the compile-time lattice size M equal to m; returns
// false for an unsupported m
template <class F>
CGP_HD inline bool lat_dispatch(int32_t m, F f) {
  switch (m) {
    case 1: f(Lat<1>{}); return true;
    case 2: f(Lat<2>{}); return true;
    case 4: f(Lat<4>{}); return true;
    case 8: f(Lat<8>{}); return true;
    default: return false;
  }
}

}  // namespace cgp

namespace cgp {

struct Hierarchy;

// Host copy of the lattice structure (built once at set-up).
struct Lattice {
  int32_t m = 1, nI = 0, nT = 0, nE = 0, nV = 0, EB = 0, VB = 0;
  std::vector<int32_t> tri_v, tri_e, edge_v, edge_t, lat_of;
  std::vector<double> af;
  std::vector<uint8_t> ldir;
  // coarse-vertex rows of the mass matrix (see LatDev): width, lattice
  // columns, and the position of each entry in the fine CSR arrays (-1 for
  // padding), from which the values are gathered once M is assembled
  int32_t vw = 0;
  std::vector<int32_t> vcol, vpos;
  std::vector<int32_t> node_of;  // [N] lattice node -> mesh node (inverse of lat_of)
  // momentum rows on the lattice (momlat.hpp): per mesh row, the CSR offset
  // of each of its six direction neighbours ([N][8], 0xff: none; rows of the
  // coarse vertices unused), and whether every row of an interior or edge
  // node matched its CSR row exactly
  std::vector<uint8_t> mslot;
  bool mom_ok = false;
  // per coarse edge, the record of its inner nodes' rows (LatEdgeRec)
  std::vector<LatEdgeRec> erec;
  // view with host pointers (vval left empty)
  LatDev host_view() const;
};

// Numbers the coarse edges (first encounter over triangles and local edges),
// maps every fine node to its lattice node and checks that the map is a
// permutation; builds the coarse-vertex rows.  Returns "" on success.
std::string build_lattice(const Hierarchy& h, Lattice& L);

// Fills L.mslot and L.mom_ok from the fine CSR graph of h.
void build_mom_slots(const Hierarchy& h, Lattice& L);

}  // namespace cgp
