// Two Chebyshev steps of the mass solves per launch over the interior lattice
// nodes (lattice size 8), for blocks of whole coarse triangles.
//
// The mass solves of Eqs. 25-26 run the Chebyshev iteration
//   x_{k+1} = x_k + ca_k (x_k - x_{k-1}) + cb_k D^-1 (b - M x_k)
// on the lattice layout (lattice.hpp).  A pair of steps runs as three
// launches: the single-step kernel computes x_{k+1} on the coarse-edge and
// vertex nodes; this kernel then computes x_{k+1} and x_{k+2} on the interior
// nodes, a block taking the interiors of kCh2Tris consecutive coarse
// triangles (a contiguous range of the layout) and reading x_k and x_{k+1}
// at the inner nodes of the triangles' edges (the only nodes outside a
// triangle's interior that its interior stencils reach); the single-step
// kernel then computes x_{k+2} on the edge and vertex nodes.  The interior
// ranges of b, x_{k-1} and x_k are read and those of x_{k+1}, x_{k+2} written
// once per two steps instead of twice.  Every value is formed with the
// operations of lat_apply in the same order.
//
// The phases are plain functions of (block, thread) over a Cheb2Shared
// workspace, so the device kernel (a barrier between phases) and a host
// emulation (each phase run for every thread before the next) run the same
// code; on the host every index is checked.
#pragma once

#include <cstdint>

#include "lattice.hpp"

namespace cgp {

constexpr int kCh2M = 8;                               // lattice size
constexpr int kCh2NI = (kCh2M - 1) * (kCh2M - 2) / 2;  // interior nodes per triangle (21)
constexpr int kCh2Tris = 12;                           // coarse triangles per block
constexpr int kCh2Own = kCh2Tris * kCh2NI;             // interior nodes per block (252)
constexpr int kCh2Halo = kCh2Tris * 3 * (kCh2M - 1);   // edge-node slots per block (252)
constexpr int kCh2All = kCh2Own + kCh2Halo;
constexpr int kCh2Threads = 256;

// set by the host emulation when an index leaves its array (one host
// thread at a time)
inline bool ch2_fault = false;
#if defined(__HIP_DEVICE_COMPILE__)
#define CH2_CHECK(c) ((void)0)
#else
#define CH2_CHECK(c) (void)(ch2_fault = ch2_fault || !(c))
#endif

// Values are stored as T (double, or float for the inner solves of the
// mixed-precision form) and combined in FP64.
//
// Block workspace (LDS on the device).  Sizes are multiples of 16 bytes, so
// every array starts 16-byte aligned when the structure does.
template <typename T, int NR>
struct Cheb2Shared {
  T xk[kCh2All * NR];  // x_k: interior nodes, then edge-node slots
  T x1[kCh2All * NR];  // x_{k+1}: interior nodes, then edge-node slots
  T xm[kCh2Own * NR];  // x_{k-1}; x_{k+2} once step 2 has run
  T b[kCh2Own * NR];   // right-hand sides
};

template <typename T>
struct Cheb2Args {
  int32_t n;    // lattice nodes
  const T* b;   // [n][NR]
  const T* xm;  // x_{k-1}
  const T* xk;  // x_k
  T* x1;        // x_{k+1}: read on the edge nodes, written on the interior
  T* x2;        // x_{k+2}, written on the interior (may be the buffer of xm)
  double ca1, cb1, ca2, cb2;
};

using Ch2Lat = Lat<kCh2M>;

CGP_HD inline int ch2_ntri(const LatDev& L, int blk) {
  const int32_t rest = L.nT - blk * kCh2Tris;
  return rest < kCh2Tris ? rest : kCh2Tris;
}

// workspace slot of point (a, b) of the block's triangle g: interior points
// in the layout's order, edge points at (3 g + j) (m - 1) + p - 1 (local
// edge j, p steps from v_j); -1 for a vertex
CGP_HD inline int ch2_slot(int g, int a, int b) {
  constexpr int M = kCh2M;
  if (a >= 1 && b >= 1 && a + b <= M - 1) return g * kCh2NI + lat_islot(M, a, b);
  if (b == 0 && a >= 1 && a <= M - 1) return kCh2Own + (g * 3 + 0) * (M - 1) + (a - 1);
  if (a + b == M && b >= 1 && b <= M - 1) return kCh2Own + (g * 3 + 1) * (M - 1) + (b - 1);
  if (a == 0 && b >= 1 && b <= M - 1) return kCh2Own + (g * 3 + 2) * (M - 1) + (M - b - 1);
  return -1;
}

// Neighbour table of the interior stencil: for each interior position r of a
// triangle (lat_islot order), the six neighbours in lat_apply's order --
// (a, b-1), (a, b+1), (a+1, b), (a+1, b-1), (a-1, b), (a-1, b+1) -- as 8-bit
// codes packed in one word: an interior position (< kCh2NI), or 32 + 7 j +
// p - 1 for the point p steps from v_j on local edge j.  Slot in a block's
// workspace for triangle g: g kCh2NI + code, plus kCh2Own - 32 for an edge
// code (the edge slots of triangle g start at kCh2Own + 3 (m - 1) g, and
// 3 (m - 1) = kCh2NI for m = 8).
struct Ch2NbTable {
  uint64_t w[kCh2NI];
};

constexpr int ch2_code(int a, int b) {
  constexpr int M = kCh2M;
  if (a >= 1 && b >= 1 && a + b <= M - 1) return lat_islot(M, a, b);
  if (b == 0) return 32 + 0 * (M - 1) + (a - 1);
  if (a + b == M) return 32 + 1 * (M - 1) + (b - 1);
  return 32 + 2 * (M - 1) + (M - b - 1);
}

constexpr Ch2NbTable ch2_make_nb_table() {
  Ch2NbTable t{};
  for (int a = 1; a <= kCh2M - 2; ++a)
    for (int b = 1; a + b <= kCh2M - 1; ++b) {
      const int pts[6][2] = {{a, b - 1}, {a, b + 1},     {a + 1, b},
                             {a + 1, b - 1}, {a - 1, b}, {a - 1, b + 1}};
      uint64_t w = 0;
      for (int q = 0; q < 6; ++q) w |= (uint64_t)ch2_code(pts[q][0], pts[q][1]) << (8 * q);
      t.w[lat_islot(kCh2M, a, b)] = w;
    }
  return t;
}

// point (a, b) of the block's triangle g held in edge-node slot h
CGP_HD inline void ch2_halo_point(int h, int& g, int& a, int& b) {
  constexpr int M = kCh2M;
  g = h / (3 * (M - 1));
  const int r = h - g * 3 * (M - 1);
  const int j = r / (M - 1), p = r - j * (M - 1) + 1;
  a = j == 0 ? p : (j == 1 ? M - p : 0);
  b = j == 0 ? 0 : (j == 1 ? p : M - p);
}

// Phase 1: the block's interior ranges of x_k, x_{k-1} and b as 16-byte
// pieces (ld16 / ldnt16 copy 16 bytes between 16-byte aligned addresses;
// ldnt16 for the streams read once), and x_k, x_{k+1} at the edge nodes.
template <typename T, int NR, class Ld16, class LdNt16>
CGP_HD inline void ch2_stage(const LatDev& L, const Cheb2Args<T>& A, int blk, int tid,
                             Cheb2Shared<T, NR>& S, Ld16 ld16, LdNt16 ldnt16) {
  constexpr int kPer = 16 / (int)sizeof(T);
  const int ntri = ch2_ntri(L, blk);
  // kCh2Own NR values per block: a multiple of 16 bytes, so aligned
  const int64_t v0 = (int64_t)blk * kCh2Own * NR;
  const int nv = ntri * kCh2NI * NR;
  CH2_CHECK(ntri > 0 && v0 + nv <= (int64_t)L.EB * NR && L.EB <= A.n);
  for (int q = tid; q * kPer < nv; q += kCh2Threads) {
    const int v = q * kPer;
    if (v + kPer <= nv) {
      ld16(A.xk + v0 + v, S.xk + v);
      ldnt16(A.xm + v0 + v, S.xm + v);
      ldnt16(A.b + v0 + v, S.b + v);
    } else {
#pragma unroll
      for (int j = 0; j < kPer; ++j)
        if (v + j < nv) {
          S.xk[v + j] = A.xk[v0 + v + j];
          S.xm[v + j] = A.xm[v0 + v + j];
          S.b[v + j] = A.b[v0 + v + j];
        }
    }
  }
  for (int h = tid; h < ntri * 3 * (kCh2M - 1); h += kCh2Threads) {
    int g, a, b;
    ch2_halo_point(h, g, a, b);
    const int32_t tri = blk * kCh2Tris + g;
    const int32_t i = Ch2Lat::index(L, tri, Ch2Lat::tri(L, tri), a, b);
    CH2_CHECK(i >= L.EB && i < L.VB && ch2_slot(g, a, b) == kCh2Own + h);
#pragma unroll
    for (int d = 0; d < NR; ++d) {
      S.xk[(kCh2Own + h) * NR + d] = A.xk[(int64_t)i * NR + d];
      S.x1[(kCh2Own + h) * NR + d] = A.x1[(int64_t)i * NR + d];
    }
  }
}

// One Chebyshev step on the block's interior nodes: reads x (current
// iterate, every slot), xm (previous, interior) and bb; writes out
// (interior).  out may be xm: a thread reads its node's xm before writing
// it, and no other thread reads that value.  nbt: the neighbour table.
template <typename T, int NR>
CGP_HD inline void ch2_step(const LatDev& L, int blk, int tid, const uint64_t* nbt,
                            const T* x, const T* xm, const T* bb, double ca, double cb, T* out) {
  const int ntri = ch2_ntri(L, blk);
  for (int t = tid; t < ntri * kCh2NI; t += kCh2Threads) {
    const int g = t / kCh2NI;
    const int r = t - g * kCh2NI;
    const double At = L.af[blk * kCh2Tris + g];
    const uint64_t w = nbt[r];
    int nb[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) {
      const int code = (int)((w >> (8 * q)) & 0xff);
      nb[q] = g * kCh2NI + code + (code >= 32 ? kCh2Own - 32 : 0);
    }
#ifndef __HIP_DEVICE_COMPILE__
    {  // host emulation: the table agrees with the points' slots
      int32_t Tq, a, b;
      Ch2Lat::interior((int32_t)r, Tq, a, b);
      const int ref[6] = {ch2_slot(g, a, b - 1),     ch2_slot(g, a, b + 1), ch2_slot(g, a + 1, b),
                          ch2_slot(g, a + 1, b - 1), ch2_slot(g, a - 1, b), ch2_slot(g, a - 1, b + 1)};
      for (int q = 0; q < 6; ++q) CH2_CHECK(nb[q] == ref[q] && nb[q] >= 0 && nb[q] < kCh2All);
      CH2_CHECK(ch2_slot(g, a, b) == t);
    }
#endif
    const bool masked = L.ldir[(int64_t)blk * kCh2Own + t] != 0;
    const double di = 1.0 / At;
#pragma unroll
    for (int d = 0; d < NR; ++d) {
      auto xq = [&](int q) { return (double)x[nb[q] * NR + d]; };
      const double s = ((xq(0) + xq(1)) + (xq(2) + xq(3))) + (xq(4) + xq(5));
      const double xv = x[t * NR + d];
      const double y = At * xv + (At / 6.0) * s;
      out[t * NR + d] = (T)((d < 2 && masked)
                                ? 0.0
                                : xv + ca * (xv - (double)xm[t * NR + d]) + cb * di * ((double)bb[t * NR + d] - y));
    }
  }
}

// Phases 2 and 3: x_{k+1} into S.x1, then x_{k+2} over S.xm.
template <typename T, int NR>
CGP_HD inline void ch2_step1(const LatDev& L, const Cheb2Args<T>& A, int blk, int tid,
                             const uint64_t* nbt, Cheb2Shared<T, NR>& S) {
  ch2_step<T, NR>(L, blk, tid, nbt, S.xk, S.xm, S.b, A.ca1, A.cb1, S.x1);
}
template <typename T, int NR>
CGP_HD inline void ch2_step2(const LatDev& L, const Cheb2Args<T>& A, int blk, int tid,
                             const uint64_t* nbt, Cheb2Shared<T, NR>& S) {
  ch2_step<T, NR>(L, blk, tid, nbt, S.x1, S.xk, S.b, A.ca2, A.cb2, S.xm);
}

// Phase 4: the interior ranges of x_{k+1} and x_{k+2} out as 16-byte pieces
// (st16 copies 16 bytes between 16-byte aligned addresses).
template <typename T, int NR, class St16>
CGP_HD inline void ch2_write(const LatDev& L, const Cheb2Args<T>& A, int blk, int tid,
                             const Cheb2Shared<T, NR>& S, St16 st16) {
  constexpr int kPer = 16 / (int)sizeof(T);
  const int ntri = ch2_ntri(L, blk);
  const int64_t v0 = (int64_t)blk * kCh2Own * NR;
  const int nv = ntri * kCh2NI * NR;
  for (int q = tid; q * kPer < nv; q += kCh2Threads) {
    const int v = q * kPer;
    if (v + kPer <= nv) {
      st16(S.x1 + v, A.x1 + v0 + v);
      st16(S.xm + v, A.x2 + v0 + v);
    } else {
#pragma unroll
      for (int j = 0; j < kPer; ++j)
        if (v + j < nv) {
          A.x1[v0 + v + j] = S.x1[v + j];
          A.x2[v0 + v + j] = S.xm[v + j];
        }
    }
  }
}

}  // namespace cgp
