// s-step ("communication-avoiding") form of the coarse Jacobi-PCG.  Internal
// to the library.
//
// Jacobi-PCG on K x = b is CG on the scaled operator A^ = D^-1/2 K D^-1/2
// (D = diag K) for x^ = D^1/2 x.  The s-step form (Chronopoulos and Gear's
// s-step CG; the stable version with a Chebyshev basis as in Carson's
// communication-avoiding Krylov methods) advances s iterations from one
// global reduction: with p^, r^ at the start of a block of s iterations,
//   V = [T_0(A^-I) p^, ..., T_s(A^-I) p^, T_0(A^-I) r^, ..., T_{s-1}(A^-I) r^]
// (Chebyshev polynomials on the spectrum [0, 2] of A^), the s CG steps are
// carried out on coefficient vectors a, c, e of length 2s+1 (p^ = V a,
// r^ = V c, x^ - x^_0 = V e) using only the Gram matrices G = V'V and
// G_D = V'DV; A^ V = V B with B the basis recurrence.  The iterates are those
// of Jacobi-PCG up to rounding, and the stopping test after every step is the
// one of the ordinary solver, ||b - K x||_2 <= tol ||b||_2 on the recursive
// residual: ||r||^2 = c' G_D c.
//
// On the GPU one launch does s iterations.  The coarse nodes are cut into
// tiles (recursive coordinate bisection); each work-group owns a tile and
// holds its depth-s neighbourhood, on which it forms the s+1 and s basis
// vectors in LDS (the matrix powers need no data from other work-groups within
// the launch).  The Gram matrices are summed over tiles by every work-group of
// the next launch in the same fixed order.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

namespace cgp {

constexpr int kCaS = 4;                     // iterations per launch
constexpr int kCaM = 2 * kCaS + 1;          // basis vectors
constexpr int kCaNU = kCaM * (kCaM + 1) / 2;  // entries of a symmetric M x M matrix
constexpr int kCaNG = 2 * kCaNU;            // G and G_D
constexpr int kCaThreads = 512;             // work-group size = most nodes a tile owns
constexpr int kCaExtMax = 1024;             // most nodes in a tile's neighbourhood
constexpr int kCaEllMax = 7680;             // most entries in a tile's ELL block (LDS)

// Host plan.  Internal node order: tile by tile, a tile's own nodes in
// ascending coarse-node order.  A tile's neighbourhood lists its own nodes,
// then the nodes at graph distance 1, 2, ..., s (each distance in ascending
// internal order).  The rows of the neighbourhood nodes at distance < s are
// stored as a local ELL block (entry k of row r at ell_off[t] + k * rows + r,
// rows = layer[t * (s + 1) + s - 1]) whose columns index the neighbourhood;
// ell_slot holds the entry's position in K's CSR arrays (-1 for padding,
// which points at the row itself with value 0).
struct CaPlan {
  int s = 0, width = 0, ntiles = 0, ntiles_pad = 0;
  int max_own = 0, max_ext = 0;
  std::vector<int32_t> perm;     // [n] internal -> coarse node
  std::vector<int32_t> own_off;  // [ntiles + 1] internal range of tile t's own nodes
  std::vector<int32_t> ext_off;  // [ntiles + 1]
  std::vector<int32_t> ext;      // neighbourhood lists, internal indices
  std::vector<int32_t> layer;    // [ntiles][s + 1]: nodes at distance <= d
  std::vector<int32_t> ell_off;  // [ntiles + 1]
  std::vector<uint16_t> ell_col;
  std::vector<int32_t> ell_slot;
};

// Builds the plan for the CSR graph (rowptr, col; every row holds its
// diagonal) with node coordinates xy [2n].  Tiles own at most own_max nodes,
// have neighbourhoods of at most ext_max nodes and ELL blocks of at most
// ell_max entries.  Returns "" or the reason it cannot.
std::string ca_plan(int32_t n, const std::vector<int32_t>& rowptr,
                    const std::vector<int32_t>& col, const double* xy, int s, int own_max,
                    int ext_max, int ell_max, CaPlan& out);

// Checks every invariant the kernels rely on (index ranges, distances,
// ownership, row contents); "" when the plan is valid.
std::string ca_check(int32_t n, const std::vector<int32_t>& rowptr,
                     const std::vector<int32_t>& col, const CaPlan& p, int own_max,
                     int ext_max, int ell_max);

// Device view of the plan and the solver's vectors (internal order).
struct CaDev {
  int32_t n = 0, ntiles = 0, ntiles_pad = 0, width = 0;
  const int32_t* perm = nullptr;
  const int32_t* own_off = nullptr;
  const int32_t* ext_off = nullptr;
  const int32_t* ext = nullptr;
  const int32_t* layer = nullptr;
  const int32_t* ell_off = nullptr;
  const uint16_t* ell_col = nullptr;
  const int32_t* ell_slot = nullptr;
  double* ell_val = nullptr;  // A^ entries
  double* sq = nullptr;       // [n] sqrt(K_ii)
  double* xh = nullptr;       // [n] x^ = D^1/2 x
  double* r0 = nullptr;       // [n] r^_0
  double* V[2] = {nullptr, nullptr};  // [2][M][n] basis at own nodes, by launch parity
  double* gpart = nullptr;    // [2][NG][ntiles_pad] Gram partials, by launch parity
  double* spart = nullptr;    // [2][ntiles_pad] ||r_0||^2, ||b||^2 partials
};

struct Scal;

// A^ entries from the assembled K (CSR values Kval, rows starting with the
// diagonal).
void launch_ca_setup(const CaDev& d, const int32_t* rowptr, const double* Kval, hipStream_t s);
// x^_0 = D^1/2 x_0, r^_0 = D^-1/2 (b - K x_0) (K x_0 from the ELL copy of K),
// partials of ||r_0||^2 and ||b||^2; resets the solver scalars.
void launch_ca_start(const CaDev& d, const int32_t* ell_col, const double* ell_val, int ell_w,
                     const double* b, const double* x, Scal* sc, hipStream_t s);
// Launch o >= 1: the s iterations (o - 2) s + 1 .. (o - 1) s (o = 1: the test
// of the guess and the first basis).
void launch_ca_outer(const CaDev& d, Scal* sc, int o, double tol, int max_iter, int my_stamp,
                     hipStream_t s, hipEvent_t* ev);
// x = D^-1/2 x^ in the caller's node order.
void launch_ca_final(const CaDev& d, double* x, hipStream_t s);

}  // namespace cgp
