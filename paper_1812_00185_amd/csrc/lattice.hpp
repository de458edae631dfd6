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
//   coarse vertex: any valence; its row of the assembled CSR matrix.
// Vectors in this layout hold, in order: the interior nodes of every coarse
// triangle (triangle-major, rows a = 1 .. m-2 of b = 1 .. m-1-a), the m - 1
// inner nodes of every coarse edge (from its lower-numbered end), the coarse
// vertices.
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
  const int32_t* rowptr;  // fine CSR (mesh numbering), rows of the coarse vertices
  const int32_t* col;
  const double* M;        // assembled fine mass matrix (vertex rows)
};

// first lattice index of interior row a (1 <= a <= m-2) within a triangle
CGP_HD inline int32_t lat_rowoff(int32_t m, int32_t a) {
  return (a - 1) * (m - 1) - ((a - 1) * a) / 2;
}

// lattice index of point (a, b) of coarse triangle T (0 <= a, b; a + b <= m)
CGP_HD inline int32_t lat_index(const LatDev& L, int32_t T, int32_t a, int32_t b) {
  const int32_t m = L.m;
  if (a >= 1 && b >= 1 && a + b <= m - 1) return T * L.nI + lat_rowoff(m, a) + (b - 1);
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

// (M x)_l for NR interleaved components (x(idx, d) reads component d of
// lattice node idx) and the diagonal M_ll
template <int NR, class X>
CGP_HD inline void lat_apply(const LatDev& L, int32_t l, X x, double (&y)[NR], double& diag) {
  const int32_t m = L.m;
  if (l < L.EB) {
    const int32_t T = l / L.nI;
    int32_t r = l - T * L.nI, a = 1;
    while (r >= m - 1 - a) {
      r -= m - 1 - a;
      ++a;
    }
    const int32_t b = r + 1;
    const int32_t nb[6] = {lat_index(L, T, a, b - 1),     lat_index(L, T, a, b + 1),
                           lat_index(L, T, a + 1, b),     lat_index(L, T, a + 1, b - 1),
                           lat_index(L, T, a - 1, b),     lat_index(L, T, a - 1, b + 1)};
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
    const int32_t E = (l - L.EB) / (m - 1);
    const int32_t t = (l - L.EB) - E * (m - 1) + 1;
    const int32_t prev = t == 1 ? L.VB + L.edge_v[2 * E] : l - 1;
    const int32_t next = t == m - 1 ? L.VB + L.edge_v[2 * E + 1] : l + 1;
    double acc[NR];
    double asum = 0.0;
#pragma unroll
    for (int d = 0; d < NR; ++d) acc[d] = 0.0;
    for (int q = 0; q < 2; ++q) {
      const int32_t tj = L.edge_t[2 * E + q];
      if (tj < 0) continue;
      const int32_t T = tj >> 2, j = tj & 3;
      const int32_t p = (L.tri_e[3 * T + j] & 1) ? m - t : t;  // steps from v_j
      int32_t i1, i2;
      if (j == 0) {
        i1 = lat_index(L, T, p, 1);
        i2 = lat_index(L, T, p - 1, 1);
      } else if (j == 1) {
        i1 = lat_index(L, T, m - p - 1, p);
        i2 = lat_index(L, T, m - p, p - 1);
      } else {
        i1 = lat_index(L, T, 1, m - p);
        i2 = lat_index(L, T, 1, m - p - 1);
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
  const int32_t v = l - L.VB;
  diag = 0.0;
#pragma unroll
  for (int d = 0; d < NR; ++d) y[d] = 0.0;
  for (int32_t s = L.rowptr[v]; s < L.rowptr[v + 1]; ++s) {
    const double mv = L.M[s];
    const int32_t c = L.col[s];
    if (c == v) diag = mv;
    const int32_t lc = L.lat_of[c];
#pragma unroll
    for (int d = 0; d < NR; ++d) y[d] += mv * x(lc, d);
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
  const int32_t v = l - L.VB;
  for (int32_t s = L.rowptr[v]; s < L.rowptr[v + 1]; ++s)
    if (L.col[s] == v) return L.M[s];
  return 0.0;
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
  // view with host pointers (CSR and M left empty)
  LatDev host_view() const;
};

// Numbers the coarse edges (first encounter over triangles and local edges),
// maps every fine node to its lattice node and checks that the map is a
// permutation.  Returns "" on success.
std::string build_lattice(const Hierarchy& h, Lattice& L);

}  // namespace cgp
