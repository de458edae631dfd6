// Momentum system of Eq. 21 on the rows of the lattice's interior and
// coarse-edge nodes, A = 3/2 M + dt nu K + dt N(w) and its right-hand side,
// with the fine geometry taken from the coarse triangles.
//
// Every fine triangle t inside a coarse triangle T = (V0, V1, V2) is T scaled
// by 1/m ("up") or its point reflection ("down"), so with T's coefficients
// B_r = Y_{r+1} - Y_{r+2}, C_r = X_{r+2} - X_{r+1} its P1 gradient
// coefficients are b_r = +-B_r / m, c_r = +-C_r / m (vertices in the roles of
// V0, V1, V2) and its area is A_t = |T| / m^2.  Per fine triangle around node
// i and each other vertex j (third vertex k):
//   M_ij += A_t / 12,  K_ij += (b_i b_j + c_i c_j) / (4 A_t),
//   N_ij += (b_j, c_j) . (2 w_i + w_j + w_k) / 24,
// the diagonal from the row sums (M_ii = sum_j M_ij, K_ii = -sum_j K_ij,
// N_ii = -sum_j N_ij), the initial residual rhs - A x0 of the BiCGSTAB solve
// (x0 = W, the boundary values on Dirichlet rows) from the row's values
// while they are in registers, and the right-hand side
//   sum_j M_ij R_j + M_ii R_i + (dt / 6) sum_t (b_i, c_i) (P_i + P_j + P_k)
// (R = 2 U^n - 1/2 U^{n-1} + dt F; the last term is -dt (G P)_i with
// G = -D^T).  An interior node of T has six neighbours, each in two of the
// six fine triangles around it; a coarse-edge node has two neighbours along
// the edge and two in each adjacent triangle (its three fine triangles per
// side taken in a frame where the edge is T's edge 0).  No coordinate, side
// or column index is read: the static slot map gives the CSR position of
// each neighbour in the row.  The rows of the coarse vertices (any valence)
// keep the side-based assembly.
//
// Plain functions of a row, shared by the device kernel and a host check.
#pragma once

#include <cstdint>

#include "lattice.hpp"

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#endif

// the per-row helpers below must inline into the kernel: passed by
// reference to an out-of-line call, their small arrays would live in scratch
#define CGP_HDI CGP_HD inline __attribute__((always_inline))

namespace cgp {

constexpr uint8_t kNoSlot = 0xff;

// The six direction points of lattice node l < VB: lattice indices, -1 where
// absent.  Interior node (a, b) of T: (a+1,b), (a,b+1), (a-1,b), (a-1,b+1),
// (a,b-1), (a+1,b-1).  Edge node (t steps from the edge's lower end): the
// neighbours at t + 1 and t - 1 along the edge, then for each adjacent
// triangle q (0, 1) the points (p, 1) and (p - 1, 1) of the frame in which
// the edge is its edge 0 and the node is (p, 0).
template <int M>
CGP_HD inline void mom_frame_point(int j, int a1, int b1, int& a, int& b) {
  if (j == 0) {
    a = a1;
    b = b1;
  } else if (j == 1) {
    a = M - a1 - b1;
    b = a1;
  } else {
    a = b1;
    b = M - a1 - b1;
  }
}

template <int M>
CGP_HD inline void mom_dirs(const LatDev& L, int32_t l, int32_t (&pt)[6]) {
  using G = Lat<M>;
  if (l < L.EB) {
    int32_t T, a, b;
    G::interior(l, T, a, b);
    const LatTri tr = G::tri(L, T);
    const int na[6] = {a + 1, a, a - 1, a - 1, a, a + 1};
    const int nb[6] = {b, b + 1, b, b + 1, b - 1, b - 1};
#pragma unroll
    for (int d = 0; d < 6; ++d) pt[d] = G::index(L, T, tr, na[d], nb[d]);
    return;
  }
  int32_t E, t;
  G::edge(L, l, E, t);
  pt[0] = t == M - 1 ? L.VB + L.edge_v[2 * E + 1] : l + 1;
  pt[1] = t == 1 ? L.VB + L.edge_v[2 * E] : l - 1;
  for (int q = 0; q < 2; ++q) {
    const int32_t tj = L.edge_t[2 * E + q];
    if (tj < 0) {
      pt[2 + 2 * q] = pt[3 + 2 * q] = -1;
      continue;
    }
    const int32_t T = tj >> 2, j = tj & 3;
    const LatTri tr = G::tri(L, T);
    const int p = (tr.te[j] & 1) ? M - t : t;
    int a, b;
    mom_frame_point<M>(j, p, 1, a, b);
    pt[2 + 2 * q] = G::index(L, T, tr, a, b);
    mom_frame_point<M>(j, p - 1, 1, a, b);
    pt[3 + 2 * q] = G::index(L, T, tr, a, b);
  }
}

// Per mesh row of an interior or coarse-edge node (built once at set-up):
// the mesh indices of its six direction neighbours (-1: none) and, per
// adjacent coarse triangle, (T << 3) | (frame j << 1) | reversed, -1 for
// none; an interior row has side 0 = T << 3 and side 1 = -2.
struct MomRow {
  int32_t nb[6];
  int32_t side[2];
};
static_assert(sizeof(MomRow) == 32, "momentum row record");

// Per coarse triangle: B_r, C_r times (orientation sign / m), the fine area.
struct MomTri {
  double B[3], C[3], At, pad;
};
static_assert(sizeof(MomTri) == 64, "momentum triangle record");

template <int M>
CGP_HD inline MomTri mom_tri_coef(const LatDev& L, const double* xy_c, int32_t T) {
  double X[3], Y[3];
  for (int r = 0; r < 3; ++r) {
    const int32_t v = L.tri_v[3 * T + r];
    X[r] = xy_c[2 * v];
    Y[r] = xy_c[2 * v + 1];
  }
  MomTri t{};
  double b0[3], c0[3];
  for (int r = 0; r < 3; ++r) {
    const int r1 = r == 2 ? 0 : r + 1, r2 = r == 0 ? 2 : r - 1;
    b0[r] = Y[r1] - Y[r2];
    c0[r] = X[r2] - X[r1];
  }
  const double a2 = b0[0] * X[0] + b0[1] * X[1] + b0[2] * X[2];
  const double sg = (a2 < 0.0 ? -1.0 : 1.0) / (double)M;
  for (int r = 0; r < 3; ++r) {
    t.B[r] = sg * b0[r];
    t.C[r] = sg * c0[r];
  }
  t.At = L.af[T];
  return t;
}

// The row record of lattice node l < VB (mesh numbering through node_of).
template <int M>
CGP_HD inline MomRow mom_row_record(const LatDev& L, const int32_t* node_of, int32_t l) {
  using G = Lat<M>;
  MomRow r;
  int32_t pt[6];
  mom_dirs<M>(L, l, pt);
  for (int d = 0; d < 6; ++d) r.nb[d] = pt[d] >= 0 ? node_of[pt[d]] : -1;
  if (l < L.EB) {
    r.side[0] = (l / L.nI) << 3;
    r.side[1] = -2;
    return r;
  }
  int32_t E, t;
  G::edge(L, l, E, t);
  for (int q = 0; q < 2; ++q) {
    const int32_t tj = L.edge_t[2 * E + q];
    if (tj < 0) {
      r.side[q] = -1;
      continue;
    }
    const int32_t T = tj >> 2, j = tj & 3;
    const LatTri tr = G::tri(L, T);
    r.side[q] = (T << 3) | (j << 1) | (tr.te[j] & 1);
  }
  return r;
}

struct MomLatArgs {
  int32_t n;                    // fine rows
  int32_t row0;                 // first row assembled here (rows below: vertex rows)
  const int32_t* rowptr;        // fine CSR (mesh numbering)
  const uint8_t* slot;          // [n][8] CSR offset in row i of direction d (kNoSlot: none)
  const MomRow* rows;           // [n] (rows from row0 on)
  const MomTri* tris;           // [nT]
  const int32_t* dir_index;     // [n] position in the Dirichlet list or -1
  const double2* W;             // [n] 2 U^n - U^{n-1}
  const double2* R;             // [n] 2 U^n - 1/2 U^{n-1} + dt F
  const double* p;              // [n] P, or nullptr (no pressure term)
  const double* udir;           // [2][ndir] Dirichlet values
  int32_t ndir;
  const double* tn;             // [2][n] traction on natural edges, or nullptr
  double dt, dtnu;
  double* A;
  double* invdA;
  double* rhs;                  // [2][n]
  double* x0;                   // [2][n]
  double* r0;                   // [2][n] the initial residual rhs - A x0
};

// Accumulators of one row: per direction M, K, N; the pressure gradient sums.
struct MomAcc {
  double m[6], k[6], nx[6];
  double gx, gy;
};

// The contributions of one fine triangle around node i.  B, C: the
// triangle's coefficients in the roles of its vertices (up/down and
// orientation signs and 1/m included); ri: role of i; the other two vertices
// in roles ra, rb are directions da, db; At: the fine area; w*, p*: w and P
// at i, a, b.
// (The directions are template arguments: the accumulators must stay in
// registers, which indexing them at run time would prevent.)
template <int DA, int DB>
CGP_HDI void mom_tri(MomAcc& s, const double (&B)[3], const double (&C)[3], int ri, int ra,
                           int rb, double At, double2 wi, double2 wa, double2 wb, double pi,
                           double pa, double pb) {
  constexpr int da = DA, db = DB;
  const double sx = 2.0 * wi.x + wa.x + wb.x, sy = 2.0 * wi.y + wa.y + wb.y;
  const double m = At * (1.0 / 12.0), i4a = 1.0 / (4.0 * At);
  s.m[da] += m;
  s.m[db] += m;
  s.k[da] += (B[ri] * B[ra] + C[ri] * C[ra]) * i4a;
  s.k[db] += (B[ri] * B[rb] + C[ri] * C[rb]) * i4a;
  s.nx[da] += (B[ra] * sx + C[ra] * sy) * (1.0 / 24.0);
  s.nx[db] += (B[rb] * sx + C[rb] * sy) * (1.0 / 24.0);
  const double ps = (pi + pa) + pb;
  s.gx += B[ri] * ps;
  s.gy += C[ri] * ps;
}

// T's coefficients in the frame rotated by j (frame role r is T's role r + j);
// the three cases written out (an index computed at run time would put t in
// scratch memory)
CGP_HDI void mom_frame_coef(const MomTri& t, int j, double (&B)[3], double (&C)[3]) {
  const double b0 = t.B[0], b1 = t.B[1], b2 = t.B[2];
  const double c0 = t.C[0], c1 = t.C[1], c2 = t.C[2];
  const bool j1 = j == 1, j2 = j == 2;
  B[0] = j1 ? b1 : (j2 ? b2 : b0);
  B[1] = j1 ? b2 : (j2 ? b0 : b1);
  B[2] = j1 ? b0 : (j2 ? b1 : b2);
  C[0] = j1 ? c1 : (j2 ? c2 : c0);
  C[1] = j1 ? c2 : (j2 ? c0 : c1);
  C[2] = j1 ? c0 : (j2 ? c1 : c2);
}

// The three fine triangles of a coarse-edge node in adjacent triangle Q, in
// the frame where the edge is its edge 0 and the node is (p, 0): up (p,0)
// (node, (p+1,0), (p,1)), up (p-1,0) ((p-1,0), node, (p-1,1)), down (p-1,0)
// ((p,1), (p-1,1), node).  The neighbour (p+1,0) is direction 0 (t + 1) or,
// on a reversed edge, 1.
template <int DP, int DM, int F1, int F2>
CGP_HDI void mom_edge_tris(MomAcc& s, const double (&B)[3], const double (&C)[3], double At,
                                 double2 wi, double pi, const double2 (&wd)[6],
                                 const double (&pd)[6]) {
  double Bm[3], Cm[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    Bm[r] = -B[r];
    Cm[r] = -C[r];
  }
  mom_tri<DP, F1>(s, B, C, 0, 1, 2, At, wi, wd[DP], wd[F1], pi, pd[DP], pd[F1]);
  mom_tri<DM, F2>(s, B, C, 1, 0, 2, At, wi, wd[DM], wd[F2], pi, pd[DM], pd[F2]);
  mom_tri<F1, F2>(s, Bm, Cm, 2, 0, 1, At, wi, wd[F1], wd[F2], pi, pd[F1], pd[F2]);
}

template <int Q, bool kTrac>
CGP_HDI void mom_edge_side(const MomLatArgs& A, const MomRow& rr, int32_t i, MomAcc& s,
                                 double2 wi, double pi, const double2 (&wd)[6],
                                 const double (&pd)[6], double& tx, double& ty) {
  const int32_t code = rr.side[Q];
  if (code < 0) return;
  const MomTri t = A.tris[code >> 3];
  const int j = (code >> 1) & 3;
  double B[3], C[3];
  mom_frame_coef(t, j, B, C);
  if (code & 1)
    mom_edge_tris<1, 0, 2 + 2 * Q, 3 + 2 * Q>(s, B, C, t.At, wi, pi, wd, pd);
  else
    mom_edge_tris<0, 1, 2 + 2 * Q, 3 + 2 * Q>(s, B, C, t.At, wi, pi, wd, pd);
  if constexpr (kTrac) {
    if (Q == 0 && rr.side[1] == -1) {
      // boundary edge, natural on a free row: its fine length from the
      // frame's edge-0 coefficients (B_2, C_2: the edge vector, scaled)
      const int64_t n = A.n;
      const double len = sqrt(B[2] * B[2] + C[2] * C[2]);
      const double ti = A.tn[i], tiy = A.tn[n + i];
      for (int d = 0; d < 2; ++d) {
        const int32_t jm = rr.nb[d];
        tx += len * (2.0 * ti + A.tn[jm]) * (1.0 / 6.0);
        ty += len * (2.0 * tiy + A.tn[n + jm]) * (1.0 / 6.0);
      }
    }
  }
}

// Assembles row i (a lattice interior or coarse-edge node, free or
// Dirichlet); its matrix values go through put(s, value) (s: CSR position).
template <bool kTrac, class Put>
CGP_HDI void mom_row(const MomLatArgs& A, int32_t i, Put put) {
  const int64_t n = A.n;
  const int32_t beg = A.rowptr[i], end = A.rowptr[i + 1];
  const int di = A.dir_index[i];
  if (di >= 0) {  // Dirichlet row: identity, right-hand side = boundary value
    for (int32_t s = beg; s < end; ++s) put(s, s == beg ? 1.0 : 0.0);
    A.invdA[i] = 1.0;
    const double gx = A.udir[di], gy = A.udir[A.ndir + di];
    A.rhs[i] = gx;
    A.rhs[n + i] = gy;
    A.x0[i] = gx;
    A.x0[n + i] = gy;
    A.r0[i] = 0.0;  // x0 holds the boundary value: no residual on this row
    A.r0[n + i] = 0.0;
    return;
  }
  const MomRow rr = A.rows[i];
  double2 wd[6];
  double pd[6];
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    const int32_t j = rr.nb[d] >= 0 ? rr.nb[d] : i;  // absent: any valid node, unused
    wd[d] = A.W[j];
    pd[d] = A.p ? A.p[j] : 0.0;
  }
  const double2 wi = A.W[i];
  const double pi = A.p ? A.p[i] : 0.0;
  MomAcc s;
#pragma unroll
  for (int d = 0; d < 6; ++d) s.m[d] = s.k[d] = s.nx[d] = 0.0;
  s.gx = s.gy = 0.0;
  double tx = 0.0, ty = 0.0;  // traction
  if (rr.side[1] == -2) {
    // interior of T: the six fine triangles up (a,b), (a-1,b), (a,b-1) and
    // down (a-1,b-1), (a,b-1), (a-1,b)
    const MomTri t = A.tris[rr.side[0] >> 3];
    double B[3], C[3], Bm[3], Cm[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      B[r] = t.B[r];
      C[r] = t.C[r];
      Bm[r] = -t.B[r];
      Cm[r] = -t.C[r];
    }
    const double At = t.At;
    mom_tri<0, 1>(s, B, C, 0, 1, 2, At, wi, wd[0], wd[1], pi, pd[0], pd[1]);
    mom_tri<2, 3>(s, B, C, 1, 0, 2, At, wi, wd[2], wd[3], pi, pd[2], pd[3]);
    mom_tri<4, 5>(s, B, C, 2, 0, 1, At, wi, wd[4], wd[5], pi, pd[4], pd[5]);
    mom_tri<2, 4>(s, Bm, Cm, 0, 1, 2, At, wi, wd[2], wd[4], pi, pd[2], pd[4]);
    mom_tri<0, 5>(s, Bm, Cm, 1, 0, 2, At, wi, wd[0], wd[5], pi, pd[0], pd[5]);
    mom_tri<1, 3>(s, Bm, Cm, 2, 0, 1, At, wi, wd[1], wd[3], pi, pd[1], pd[3]);
  } else {
    // coarse-edge node: three fine triangles per adjacent coarse triangle, in
    // the frame where the edge is its edge 0 and the node is (p, 0): up (p,0)
    // (node, (p+1,0), (p,1)), up (p-1,0) ((p-1,0), node, (p-1,1)), down
    // (p-1,0) ((p,1), (p-1,1), node)
    mom_edge_side<0, kTrac>(A, rr, i, s, wi, pi, wd, pd, tx, ty);
    mom_edge_side<1, kTrac>(A, rr, i, s, wi, pi, wd, pd, tx, ty);
  }
  const uint8_t* sl = A.slot + 8 * (int64_t)i;
  double sm = 0.0, sk = 0.0, sn = 0.0, rx = 0.0, ry = 0.0, ax = 0.0, ay = 0.0;
#pragma unroll
  for (int d = 0; d < 6; ++d) {
    if (sl[d] == kNoSlot) continue;
    const double av = 1.5 * s.m[d] + A.dtnu * s.k[d] + A.dt * s.nx[d];
    put(beg + sl[d], av);
    sm += s.m[d];
    sk += s.k[d];
    sn += s.nx[d];
    const int32_t j = rr.nb[d];
    const double2 rj = A.R[j];  // R only here: fewer live registers
    rx += s.m[d] * rj.x;
    ry += s.m[d] * rj.y;
    // (A x0) at this row: x0 = W, the boundary value on Dirichlet rows
    const int dj = A.dir_index[j];
    ax += av * (dj >= 0 ? A.udir[dj] : wd[d].x);
    ay += av * (dj >= 0 ? A.udir[A.ndir + dj] : wd[d].y);
  }
  const double2 ri = A.R[i];
  const double aii = 1.5 * sm - A.dtnu * sk - A.dt * sn;
  put(beg, aii);
  A.invdA[i] = 1.0 / aii;
  rx += sm * ri.x + (A.dt / 6.0) * s.gx;
  ry += sm * ri.y + (A.dt / 6.0) * s.gy;
  if constexpr (kTrac) {
    rx += A.dt * tx;
    ry += A.dt * ty;
  }
  A.rhs[i] = rx;
  A.rhs[n + i] = ry;
  A.x0[i] = wi.x;
  A.x0[n + i] = wi.y;
  A.r0[i] = rx - (aii * wi.x + ax);
  A.r0[n + i] = ry - (aii * wi.y + ay);
}

}  // namespace cgp
