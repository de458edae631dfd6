// Right-hand sides of the mass solves of Eqs. 25-26 on the lattice layout:
//   velocity  -(2/3) dt G phi_f  (0 on velocity-Dirichlet rows)
//   pressure  -nu D U~           (rotational form, chi = 1)
// with G = -D^T and (D U)_i = int psi_i div U_h, element by element over the
// fine triangles: a fine triangle t contributes -b_i^t (phi_1 + phi_2 +
// phi_3) / 6 to (G phi)_i and sum_v (b_v^t u_v + c_v^t v_v) / 6 to (D U)_i,
// (b^t, c^t) the P1 gradient coefficients of t (areas cancel).
//
// Inside a coarse triangle T = (V0, V1, V2) every fine triangle is T scaled
// by 1/m ("up", vertices (a,b), (a+1,b), (a,b+1) in the roles of V0, V1, V2)
// or its point reflection ("down", vertices (a+1,b+1), (a,b+1), (a+1,b) in
// those roles), so b^t = +-B_r / m, c^t = +-C_r / m with T's coefficients
// B_r = Y_{r+1} - Y_{r+2}, C_r = X_{r+2} - X_{r+1}: no fine coordinate is
// read.  At a node interior to T the six triangles around it collapse to a
// stencil over its six neighbours whose weights are differences of T's
// coefficients (its own value cancels); at a node on a coarse edge or a
// coarse vertex the fine triangles around it are summed one by one, which
// keeps the boundary terms of the weak gradient.  U~ (and phi_f) are read
// from a lattice-ordered copy that a pass through the lattice-to-mesh map
// writes first, so that a stencil reads its neighbours from one array in
// lattice order.  When phi_f is known to be the prolongation of phi_c (Eq.
// 24: P1 on the coarse triangles), phi at a lattice point is interpolated
// from T's three coarse values instead, the interior gradient collapses to
// -6 sgn(T) sum_r B_r phi_r / m^2, and the copy holds (u, v) only.
//
// Plain functions of a lattice node, shared by the device kernel and a host
// check.
#pragma once

#include <cstdint>

#include "lattice.hpp"

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#endif

namespace cgp {

// set by the host check when an index leaves its array (one host thread at
// a time)
inline bool corr_fault = false;
#if defined(__HIP_DEVICE_COMPILE__)
#define CORR_CHECK(c) ((void)0)
#else
#define CORR_CHECK(c) (void)(corr_fault = corr_fault || !(c))
#endif

struct CorrLatArgs {
  int32_t n;               // fine nodes
  const double* xy_c;      // [2 N_c] coarse coordinates, interleaved
  const int32_t* cn_ptr;   // [N_c + 1] coarse node -> (triangle << 2 | role)
  const int32_t* cn_tri;
  // per lattice node (phi_f, u~, v~, 0) ([n][4]), or (u~, v~) ([n][2]) when
  // phi_c is given
  const double* v4;
  const double* phi_c;     // [N_c] coarse phi, or nullptr
  double dt, nu;
  int chi;
};

// the inputs in lattice order, i = node_of[l]: v4[l] = (phi[i], ut[i],
// ut[n + i], 0), or (ut[i], ut[n + i]) when phi is nullptr
CGP_HD inline void corr_gather(int32_t n, const int32_t* node_of, const double* phi,
                               const double* ut, int32_t l, double* v4) {
  const int32_t i = node_of[l];
  CORR_CHECK(i >= 0 && i < n);
  if (phi) {
    v4[4 * (int64_t)l] = phi[i];
    v4[4 * (int64_t)l + 1] = ut[i];
    v4[4 * (int64_t)l + 2] = ut[(int64_t)n + i];
    v4[4 * (int64_t)l + 3] = 0.0;
  } else {
    v4[2 * (int64_t)l] = ut[i];
    v4[2 * (int64_t)l + 1] = ut[(int64_t)n + i];
  }
}

struct CorrTri {
  double B[3], C[3];
  double s;  // sign of T's orientation / m
};

template <int M>
CGP_HD inline CorrTri corr_tri(const LatDev& L, const CorrLatArgs& A, int32_t T) {
  double X[3], Y[3];
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int32_t v = L.tri_v[3 * T + r];
    X[r] = A.xy_c[2 * v];
    Y[r] = A.xy_c[2 * v + 1];
  }
  CorrTri g;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const int r1 = r == 2 ? 0 : r + 1, r2 = r == 0 ? 2 : r - 1;
    g.B[r] = Y[r1] - Y[r2];
    g.C[r] = X[r2] - X[r1];
  }
  const double a2 = g.B[0] * X[0] + g.B[1] * X[1] + g.B[2] * X[2];  // twice the signed area
  g.s = (a2 < 0.0 ? -1.0 : 1.0) / (double)M;
  return g;
}

// u, v (and phi unless kPc) at lattice node l
template <bool kPc>
CGP_HD inline void corr_val(const CorrLatArgs& A, int32_t l, double& ph, double& u, double& v) {
  CORR_CHECK(l >= 0 && l < A.n);
  if constexpr (kPc) {
    const double2 q = reinterpret_cast<const double2*>(A.v4)[l];
    u = q.x;
    v = q.y;
  } else {
    const double2* q = reinterpret_cast<const double2*>(A.v4) + 2 * (int64_t)l;
    const double2 q0 = q[0], q1 = q[1];
    ph = q0.x;
    u = q0.y;
    v = q1.x;
  }
}

// the coarse phi at T's vertices (kPc)
CGP_HD inline void corr_phic(const LatDev& L, const CorrLatArgs& A, int32_t T, double (&pc)[3]) {
#pragma unroll
  for (int r = 0; r < 3; ++r) pc[r] = A.phi_c[L.tri_v[3 * T + r]];
}

// acc += contributions of the fine triangles of T around its point (a, b):
// acc[0], acc[1] = sum_t b_i^t, c_i^t (phi_1 + phi_2 + phi_3) and acc[2] =
// sum_t sum_v (b_v^t u_v + c_v^t v_v), orientation included.
template <int M, bool kPc>
CGP_HD inline void corr_around(const LatDev& L, const CorrLatArgs& A, int32_t T, int a, int b,
                               double (&acc)[3]) {
  using G = Lat<M>;
  const LatTri tr = G::tri(L, T);
  const CorrTri g = corr_tri<M>(L, A, T);
  double pc[3] = {0.0, 0.0, 0.0};
  if constexpr (kPc) corr_phic(L, A, T, pc);
  // the six candidate triangles: corner point (a0, b0), up or down, and the
  // role of (a, b) in it
  const int ca[6] = {a, a - 1, a, a - 1, a, a - 1};
  const int cb[6] = {b, b, b - 1, b - 1, b - 1, b};
  const bool up[6] = {true, true, true, false, false, false};
  const int role[6] = {0, 1, 2, 0, 1, 2};
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int a0 = ca[q], b0 = cb[q];
    const bool exists = a0 >= 0 && b0 >= 0 && (up[q] ? a0 + b0 <= M - 1 : a0 + b0 <= M - 2);
    if (!exists) continue;
    // vertices in the roles of V0, V1, V2
    int pa[3], pb[3];
    if (up[q]) {
      pa[0] = a0; pb[0] = b0; pa[1] = a0 + 1; pb[1] = b0; pa[2] = a0; pb[2] = b0 + 1;
    } else {
      pa[0] = a0 + 1; pb[0] = b0 + 1; pa[1] = a0; pb[1] = b0 + 1; pa[2] = a0 + 1; pb[2] = b0;
    }
    double ph[3], u[3], v[3];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      corr_val<kPc>(A, G::index(L, T, tr, pa[r], pb[r]), ph[r], u[r], v[r]);
      if constexpr (kPc)  // P1 on T (Eq. 24)
        ph[r] = (pc[0] * (double)(M - pa[r] - pb[r]) + pc[1] * (double)pa[r] + pc[2] * (double)pb[r]) *
                (1.0 / (double)M);
    }
    const double s = up[q] ? g.s : -g.s;
    const double sp = (ph[0] + ph[1]) + ph[2];
    acc[0] += s * g.B[role[q]] * sp;
    acc[1] += s * g.C[role[q]] * sp;
    acc[2] += s * (((g.B[0] * u[0] + g.B[1] * u[1]) + g.B[2] * u[2]) +
                   ((g.C[0] * v[0] + g.C[1] * v[1]) + g.C[2] * v[2]));
  }
}

// The right-hand sides at lattice node l: out[0], out[1] velocity, out[2]
// pressure (chi = 1).
template <int M, bool kPc>
CGP_HD inline void corr_node(const LatDev& L, const CorrLatArgs& A, int32_t l, double (&out)[3]) {
  using G = Lat<M>;
  double acc[3] = {0.0, 0.0, 0.0};
  if (l < L.EB) {
    // interior of T: the stencil over the six neighbours, weights
    // differences of T's coefficients; neighbour order (a+1,b), (a,b+1),
    // (a-1,b), (a-1,b+1), (a,b-1), (a+1,b-1)
    int32_t T, a, b;
    G::interior(l, T, a, b);
    const LatTri tr = G::tri(L, T);
    const CorrTri g = corr_tri<M>(L, A, T);
    const int na[6] = {a + 1, a, a - 1, a - 1, a, a + 1};
    const int nb[6] = {b, b + 1, b, b + 1, b - 1, b - 1};
    // (D U) weights: B_1 - B_0, B_2 - B_0, B_0 - B_1, B_2 - B_1, B_0 - B_2,
    // B_1 - B_2 (and C likewise); (G phi) weights their negatives
    const int wp[6] = {1, 2, 0, 2, 0, 1}, wm[6] = {0, 0, 1, 1, 2, 2};
    double gx = 0.0, gy = 0.0, dv = 0.0;
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      double ph = 0.0, u, v;
      corr_val<kPc>(A, G::index(L, T, tr, na[q], nb[q]), ph, u, v);
      const double wb = g.B[wp[q]] - g.B[wm[q]], wc = g.C[wp[q]] - g.C[wm[q]];
      if constexpr (!kPc) {
        gx -= wb * ph;
        gy -= wc * ph;
      }
      dv += wb * u + wc * v;
    }
    if constexpr (kPc) {  // phi linear on T: the stencil sums to -6 sum_r B_r phi_r / m
      double pc[3];
      corr_phic(L, A, T, pc);
      gx = -6.0 * ((g.B[0] * pc[0] + g.B[1] * pc[1]) + g.B[2] * pc[2]) * (1.0 / (double)M);
      gy = -6.0 * ((g.C[0] * pc[0] + g.C[1] * pc[1]) + g.C[2] * pc[2]) * (1.0 / (double)M);
    }
    acc[0] = g.s * gx;
    acc[1] = g.s * gy;
    acc[2] = g.s * dv;
  } else if (l < L.VB) {
    int32_t E, t;
    G::edge(L, l, E, t);
    for (int q = 0; q < 2; ++q) {
      const int32_t tj = L.edge_t[2 * E + q];
      if (tj < 0) continue;
      const int32_t T = tj >> 2;
      int32_t a, b;
      G::edge_point(G::tri(L, T), tj & 3, t, a, b);
      corr_around<M, kPc>(L, A, T, a, b, acc);
    }
  } else {
    const int32_t vtx = l - L.VB;
    for (int32_t k = A.cn_ptr[vtx]; k < A.cn_ptr[vtx + 1]; ++k) {
      const int32_t T = A.cn_tri[k] >> 2, r = A.cn_tri[k] & 3;
      corr_around<M, kPc>(L, A, T, r == 1 ? M : 0, r == 2 ? M : 0, acc);
    }
  }
  const bool dir = L.ldir[l] != 0;
  out[0] = dir ? 0.0 : (A.dt / 9.0) * acc[0];
  out[1] = dir ? 0.0 : (A.dt / 9.0) * acc[1];
  out[2] = A.chi ? -A.nu * acc[2] * (1.0 / 6.0) : 0.0;
}

}  // namespace cgp
