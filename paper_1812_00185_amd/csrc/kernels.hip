// HIP kernels of the CGP step for gfx950 (wave64).
//
// Operators are assembled from the CSR node graph with "edge sides" (for an
// off-diagonal slot (i, j): the third vertex of each triangle sharing edge
// ij, with its orientation).  For P1 triangles every per-row quantity follows
// from the sides of the row:
//   with (i, j, k) taken counter-clockwise (sign s = +1 for the ccw side,
//   -1 for the cw side), |e| = s det(x_j - x_i, x_k - x_i) / 2 and
//   b_i = s (y_j - y_k), c_i = s (x_k - x_j), b_j = s (y_k - y_i), c_j = s (x_i - x_k):
//     mass        M_ij  = sum |e| / 12,          M_ii = sum_j M_ij
//     stiffness   K_ij  = sum (b_i b_j + c_i c_j) / (4|e|),  K_ii = -sum_j K_ij
//     convection  N_ij  = sum ((2 w_i + w_j + w_k) . (b_j, c_j)) / 24,  N_ii = -sum_j N_ij
//     divergence  (D u)_i = sum_sides (b_j u_j + c_j v_j) / 6 + (b_i u_i + c_i v_i) / 12
//     gradient    (G p)_i = -sum_sides (b_i, c_i) (p_j + p_i / 2) / 6      (G = -D^T)
// (each triangle at i appears as two sides of row i).  No element matrices are
// stored and no atomics are used: every output row is owned by one thread or
// one lane group, and every reduction is a fixed-order two-pass block sum, so
// results are bitwise reproducible run to run.
//
// Sparse products stage a row tile (<= 256 rows, <= kTileNnz nonzeros) of the
// CSR values and columns in LDS with coalesced loads, then one thread per row
// gathers the vector; this keeps many full cache lines in flight per CU.
#include <cmath>

#include "cgp.h"
#include "device.hpp"
#include "momlat.hpp"
#include "mesh.hpp"
#include "mpnn.hpp"

namespace cgp {
namespace {

constexpr int kWaves = kBlock / 64;
static_assert(kTileRows == kBlock, "one thread per tile row");

// reduction slot kinds (x2 right-hand sides)
enum { SL_RR = 0, SL_RZ = 1, SL_BB = 2, SL_PQ = 3, SL_RHR = 4, SL_RHV = 5, SL_SS = 6, SL_TS = 7 };
// BiCGSTAB's (t, t) reuses the PQ slot
#define SL_TT SL_PQ

__device__ __forceinline__ int slot(int kind, int d) { return (kind * 2 + d) * kNbMax; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum NS per-thread values over the block; thread 0 stores them at
// part[idx[s] + blockIdx.x].
template <int NS>
__device__ void block_store(const double (&v)[NS], double* part, const int (&idx)[NS]) {
  __shared__ double sh[NS][kWaves];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const double t = wave_sum(v[s]);
    if (lane == 0) sh[s][wv] = t;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      double t = 0.0;
      for (int w = 0; w < kWaves; ++w) t += sh[s][w];
      part[idx[s] + blockIdx.x] = t;
    }
  }
}

// Every thread of the block receives sum_{b < nb} part[idx[s] + b], summed in
// the same order by every block.
template <int NS>
__device__ void block_sums(const double* part, int nb, const int (&idx)[NS], double (&out)[NS]) {
  __shared__ double sh[NS][kWaves];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // every load of every sum is issued before the first reduction (nb <= kNbMax)
  double t[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) t[s] = 0.0;
#pragma unroll
  for (int q = 0; q < kNbMax / kBlock; ++q) {
    const int b = threadIdx.x + q * kBlock;
    if (b < nb) {
#pragma unroll
      for (int s = 0; s < NS; ++s) t[s] += part[idx[s] + b];
    }
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const double v = wave_sum(t[s]);
    if (lane == 0) sh[s][wv] = v;
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    double t = 0.0;
    for (int w = 0; w < kWaves; ++w) t += sh[s][w];
    out[s] = t;
  }
  __syncthreads();
}

__device__ __forceinline__ bool active(const Scal* sc, int d, int my_stamp) {
  const int st = sc[d].done_stamp;
  return st == 0 || st >= my_stamp;
}

__device__ __forceinline__ void reset_scal(Scal& s) {
  s.rho[0] = s.rho[1] = 0.0;
  s.rho_old = s.alpha = s.omega = 1.0;
  s.bb = 0.0;
  s.rel = 0.0;
  s.done_stamp = 0;
  s.iters = 0;
  s.status = 0;
}

// LDS stage of one row tile of a CSR matrix.
template <typename T>
struct TileStage {
  T val[kTileNnz];
  int32_t col[kTileNnz];
};

// Loads the nonzeros of rows [r0, r1) into LDS (coalesced); returns the first
// nonzero index s0.  Brackets the stage with barriers so a block can loop over
// tiles.
// kStream: the matrix is streamed once per launch (the fine momentum matrix,
// hundreds of MB): its values and column indices are loaded non-temporally
// so that the L2 keeps the gathered vector; the coarse matrices, re-read by
// every iteration from cache, load normally.
template <typename T, bool kStream = false>
__device__ __forceinline__ int stage_tile(TileStage<T>& st, const DLevel& L, const T* __restrict__ val,
                                          int r0, int r1) {
  const int s0 = L.rowptr[r0], s1 = L.rowptr[r1];
  __syncthreads();
#pragma unroll 4
  for (int k = threadIdx.x; k < s1 - s0; k += kBlock) {
    if constexpr (kStream) {
      st.val[k] = __builtin_nontemporal_load(val + s0 + k);
      st.col[k] = __builtin_nontemporal_load(L.col + s0 + k);
    } else {
      st.val[k] = val[s0 + k];
      st.col[k] = L.col[s0 + k];
    }
  }
  __syncthreads();
  return s0;
}

constexpr int kRowBatch = 8;   // gathers of a row issued together
static_assert(kRowBatch == kEllPad, "ELL width padding matches the gather batch");

// acc[d] = sum over the staged nonzeros [a, b) of val * g(d, col), the
// gathers of up to kRowBatch nonzeros in flight at once (in order, so the
// summation order is that of the row).
template <typename T, int NR, class G>
__device__ __forceinline__ void tile_row_range(const TileStage<T>& st, int a, int b, G g,
                                               T (&acc)[NR]) {
#pragma unroll
  for (int d = 0; d < NR; ++d) acc[d] = T(0);
  for (int s = a; s < b; s += kRowBatch) {
    T v[kRowBatch];
    T x[kRowBatch][NR];
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) {
      if (s + u < b) {
        v[u] = st.val[s + u];
        const int c = st.col[s + u];
#pragma unroll
        for (int d = 0; d < NR; ++d) x[u][d] = g(d, c);
      }
    }
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u)
      if (s + u < b) {
#pragma unroll
        for (int d = 0; d < NR; ++d) acc[d] += v[u] * x[u][d];
      }
  }
}

template <typename T, int NR, class G>
__device__ __forceinline__ void tile_row(const TileStage<T>& st, const DLevel& L, int s0, int row,
                                         G g, T (&acc)[NR]) {
  tile_row_range<T, NR>(st, L.rowptr[row] - s0, L.rowptr[row + 1] - s0, g, acc);
}

// tile_row for two right-hand sides stored interleaved ([n][2]): one
// 16-byte gather per nonzero
__device__ __forceinline__ void tile_row2(const TileStage<double>& st, const DLevel& L, int s0,
                                          int row, const double2* __restrict__ x2,
                                          double (&acc)[2]) {
  const int a = L.rowptr[row] - s0, b = L.rowptr[row + 1] - s0;
  acc[0] = acc[1] = 0.0;
  for (int s = a; s < b; s += kRowBatch) {
    double v[kRowBatch];
    double2 x[kRowBatch];
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) {
      if (s + u < b) {
        v[u] = st.val[s + u];
        x[u] = x2[st.col[s + u]];
      }
    }
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u)
      if (s + u < b) {
        acc[0] += v[u] * x[u].x;
        acc[1] += v[u] * x[u].y;
      }
  }
}

struct SideGeo {
  double area, bi, ci, bj, cj;
};

__device__ __forceinline__ SideGeo side_geo(double2 pi, double2 pj, double2 pk, double sg) {
  SideGeo g;
  const double a2 = (pj.x - pi.x) * (pk.y - pi.y) - (pk.x - pi.x) * (pj.y - pi.y);
  g.area = 0.5 * sg * a2;
  g.bi = sg * (pj.y - pk.y);
  g.ci = sg * (pk.x - pj.x);
  g.bj = sg * (pk.y - pi.y);
  g.cj = sg * (pi.x - pk.x);
  return g;
}

constexpr int kRowLanes = 4;   // lanes per row in the side-based row kernels (rows of 7 entries)

template <int NS>
__device__ __forceinline__ void group_sum(double (&v)[NS]) {
#pragma unroll
  for (int o = kRowLanes / 2; o > 0; o >>= 1)
#pragma unroll
    for (int s = 0; s < NS; ++s) v[s] += __shfl_xor(v[s], o, kRowLanes);
}

// ------------------------------------------------------------------ assembly

__global__ void __launch_bounds__(kBlock)
k_mass_assemble(DLevel L, double* __restrict__ Mval) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < L.n; i += gridDim.x * blockDim.x) {
    const int beg = L.rowptr[i], end = L.rowptr[i + 1];
    const double2 pi = L.xy[i];
    double dm = 0.0;
    for (int s = beg + 1; s < end; ++s) {
      const double2 pj = L.xy[L.col[s]];
      double m = 0.0;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int k = L.side[2 * s + q];
        if (k < 0) continue;
        m += side_geo(pi, pj, L.xy[k], q == 0 ? 1.0 : -1.0).area * (1.0 / 12.0);
      }
      Mval[s] = m;
      dm += m;
    }
    Mval[beg] = dm;
  }
}

__global__ void __launch_bounds__(kBlock)
k_coarse_assemble(DLevel L, const uint8_t* __restrict__ nat, double* __restrict__ Kval,
                  float* __restrict__ Kval32, double* __restrict__ Dx, double* __restrict__ Dy,
                  double* __restrict__ invd, float* __restrict__ invd32,
                  double* __restrict__ lumped) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < L.n; i += gridDim.x * blockDim.x) {
    const int beg = L.rowptr[i], end = L.rowptr[i + 1];
    const double2 pi = L.xy[i];
    const bool nat_i = nat[i] != 0;
    double dk = 0.0, dxi = 0.0, dyi = 0.0, lump = 0.0;
    for (int s = beg + 1; s < end; ++s) {
      const int j = L.col[s];
      const double2 pj = L.xy[j];
      double kk = 0.0, dx = 0.0, dy = 0.0;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        const int k = L.side[2 * s + q];
        if (k < 0) continue;
        const SideGeo g = side_geo(pi, pj, L.xy[k], q == 0 ? 1.0 : -1.0);
        kk += (g.bi * g.bj + g.ci * g.cj) / (4.0 * g.area);
        dx += g.bj * (1.0 / 6.0);
        dy += g.cj * (1.0 / 6.0);
        dxi += g.bi * (1.0 / 12.0);
        dyi += g.ci * (1.0 / 12.0);
        lump += g.area * (1.0 / 6.0);
      }
      dk += kk;
      // phi = 0 rows and columns removed: identity rows, zero coupling
      const double kv = (nat_i || nat[j]) ? 0.0 : kk;
      Kval[s] = kv;
      Kval32[s] = (float)kv;
      Dx[s] = dx;
      Dy[s] = dy;
    }
    const double kii = nat_i ? 1.0 : -dk;
    Kval[beg] = kii;
    Kval32[beg] = (float)kii;
    invd[i] = 1.0 / kii;
    invd32[i] = (float)(1.0 / kii);
    Dx[beg] = dxi;
    Dy[beg] = dyi;
    lumped[i] = lump;
  }
}


// Momentum matrix A = 3/2 M + dt nu K + dt N(w), w = 2 U^n - U^{n-1}, and the
// right-hand side -dt G P + M (2 U^n - 1/2 U^{n-1} + dt F) (Eq. 21), one lane
// group per row, one lane per off-diagonal slot; Dirichlet rows become
// identity rows with the boundary value as right-hand side and as initial
// guess.
// Per node, the two fields the assembly gathers at neighbours, as pairs:
// W = 2 U^n - U^{n-1} (convecting velocity) and R = 2 U^n - 1/2 U^{n-1} + dt F
// (the mass-weighted right-hand-side field), so a neighbour costs two 16-byte
// loads instead of six 8-byte ones.
__global__ void k_momentum_fields(int32_t n32, const double* __restrict__ up,
                                  const double* __restrict__ u, const double* __restrict__ f,
                                  double dt, double2* __restrict__ W, double2* __restrict__ R) {
  const int64_t n = n32;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const double ux = u[i], uy = u[n + i], px = up[i], py = up[n + i];
    double rx = 2.0 * ux - 0.5 * px, ry = 2.0 * uy - 0.5 * py;
    if (f) {
      rx += dt * f[i];
      ry += dt * f[n + i];
    }
    W[i] = make_double2(2.0 * ux - px, 2.0 * uy - py);
    R[i] = make_double2(rx, ry);
  }
}

// kTrac: the traction t_N of Eq. 11 (nodal values tn [2][N]) on the natural
// edges adds dt int_{Gamma_N} t_h psi_i ds to the right-hand side.  On a free
// row every boundary slot (i, j) (an edge with one side missing) is a
// natural edge, since a node on a Dirichlet edge is a Dirichlet row; on an
// edge of length l the P1 boundary mass gives l (2 t_i + t_j) / 6.
// Rows [0, row_end), by blocks blk, blk + nblk, ... of kBlock / kRowLanes
// rows each.
template <bool kTrac>
__device__ __forceinline__ void mom_side_rows(
    const DLevel& L, int32_t row_end, const int32_t* __restrict__ dir_index, double dt,
    double dtnu, const double2* __restrict__ W, const double2* __restrict__ R,
    const double* __restrict__ p, const double* __restrict__ udir, int32_t ndir,
    const double* __restrict__ tn, double* __restrict__ A, double* __restrict__ invdA,
    double* __restrict__ rhs, double* __restrict__ x0, double* __restrict__ r0, int blk,
    int nblk) {
  const int64_t n = L.n;
  const int lane = threadIdx.x % kRowLanes, rpb = kBlock / kRowLanes;
  for (int base = blk * rpb; base < row_end; base += nblk * rpb) {
    const int i = base + threadIdx.x / kRowLanes;
    if (i >= row_end) continue;  // uniform within the lane group
    const int beg = L.rowptr[i], end = L.rowptr[i + 1];
    const int di = dir_index[i];
    if (di >= 0) {  // Dirichlet row: identity, right-hand side = boundary value
      for (int s = beg + lane; s < end; s += kRowLanes) A[s] = s == beg ? 1.0 : 0.0;
      if (lane == 0) {
        invdA[i] = 1.0;
        const double gx = udir[di], gy = udir[ndir + di];
        rhs[i] = gx;
        rhs[n + i] = gy;
        // the initial guess satisfies the Dirichlet condition exactly, so these
        // rows keep a zero residual and BiCGSTAB works on the free rows only
        x0[i] = gx;
        x0[n + i] = gy;
        r0[i] = 0.0;
        r0[n + i] = 0.0;
      }
      continue;
    }
    const double2 pi = L.xy[i];
    // p == nullptr: no pressure term (the non-incremental scheme)
    const double Pi = p ? p[i] : 0.0;
    const double2 wi = W[i];
    const double wix = wi.x, wiy = wi.y;
    // dm, dk, dn, rx, ry, gx, gy (, tx, ty: traction), then (A x0)_i without
    // the diagonal term
    constexpr int NA = (kTrac ? 9 : 7) + 2, AX = NA - 2;
    double acc[NA];
#pragma unroll
    for (int q = 0; q < NA; ++q) acc[q] = 0.0;
    // Every gather of a slot (node j and both side vertices) is issued before
    // any arithmetic -- a missing side reads node j instead and its terms are
    // skipped -- so a slot waits for two memory round trips (the column and
    // sides, then the node data) instead of one per side.
    struct Slot {
      int j;
      int2 sd;
      double2 pj, wj, rj, pk[2], wk[2], xj;
      double Pj, tj[2];
    };
    const int2* side2 = reinterpret_cast<const int2*>(L.side);
    auto load = [&](int s, Slot& d) {
      d.j = L.col[s];
      d.sd = side2[s];
      const int j = d.j;
      const int k0 = d.sd.x >= 0 ? d.sd.x : j, k1 = d.sd.y >= 0 ? d.sd.y : j;
      d.pj = L.xy[j];
      d.wj = W[j];
      d.rj = R[j];
      // the initial guess at j: W, or the boundary value on a Dirichlet row
      const int dj = dir_index[j];
      d.xj = dj >= 0 ? make_double2(udir[dj], udir[ndir + dj]) : d.wj;
      d.Pj = p ? p[j] : 0.0;
      d.pk[0] = L.xy[k0];
      d.wk[0] = W[k0];
      d.pk[1] = L.xy[k1];
      d.wk[1] = W[k1];
      if constexpr (kTrac) {
        d.tj[0] = tn[j];
        d.tj[1] = tn[n + j];
      }
    };
    auto add = [&](int s, const Slot& d) {
      const double2 pj = d.pj;
      if constexpr (kTrac) {
        if (d.sd.x < 0 || d.sd.y < 0) {  // boundary edge: natural on a free row
          const double l = sqrt((pj.x - pi.x) * (pj.x - pi.x) + (pj.y - pi.y) * (pj.y - pi.y));
          acc[7] += l * (2.0 * tn[i] + d.tj[0]) * (1.0 / 6.0);
          acc[8] += l * (2.0 * tn[n + i] + d.tj[1]) * (1.0 / 6.0);
        }
      }
      const double wjx = d.wj.x, wjy = d.wj.y;
      const double Pj = d.Pj;
      double m = 0.0, kk = 0.0, nn = 0.0;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if ((q == 0 ? d.sd.x : d.sd.y) < 0) continue;
        const SideGeo g = side_geo(pi, pj, d.pk[q], q == 0 ? 1.0 : -1.0);
        const double wkx = d.wk[q].x, wky = d.wk[q].y;
        m += g.area * (1.0 / 12.0);
        kk += (g.bi * g.bj + g.ci * g.cj) / (4.0 * g.area);
        nn += ((2.0 * wix + wjx + wkx) * g.bj + (2.0 * wiy + wjy + wky) * g.cj) * (1.0 / 24.0);
        acc[5] += g.bi * (Pj + 0.5 * Pi);
        acc[6] += g.ci * (Pj + 0.5 * Pi);
      }
      const double av = 1.5 * m + dtnu * kk + dt * nn;
      A[s] = av;
      acc[AX] += av * d.xj.x;
      acc[AX + 1] += av * d.xj.y;
      acc[0] += m;
      acc[1] += kk;
      acc[2] += nn;
      acc[3] += m * d.rj.x;
      acc[4] += m * d.rj.y;
    };
    for (int s = beg + 1 + lane; s < end; s += kRowLanes) {
      Slot a;
      load(s, a);
      add(s, a);
    }
    group_sum<NA>(acc);
    if (lane == 0) {
      const double2 ri = R[i];
      const double bxi = ri.x, byi = ri.y;
      const double aii = 1.5 * acc[0] - dtnu * acc[1] - dt * acc[2];
      A[beg] = aii;
      invdA[i] = 1.0 / aii;
      double rx = acc[3] + acc[0] * bxi + (dt / 6.0) * acc[5];
      double ry = acc[4] + acc[0] * byi + (dt / 6.0) * acc[6];
      if constexpr (kTrac) {
        rx += dt * acc[7];
        ry += dt * acc[8];
      }
      rhs[i] = rx;
      rhs[n + i] = ry;
      x0[i] = wix;
      x0[n + i] = wiy;
      r0[i] = rx - (aii * wix + acc[AX]);
      r0[n + i] = ry - (aii * wiy + acc[AX + 1]);
    }
  }
}

template <bool kTrac>
__global__ void __launch_bounds__(kBlock)
k_momentum_assemble(DLevel L, const int32_t* __restrict__ dir_index, double dt, double dtnu,
                    const double2* __restrict__ W, const double2* __restrict__ R,
                    const double* __restrict__ p, const double* __restrict__ udir, int32_t ndir,
                    const double* __restrict__ tn, double* __restrict__ A,
                    double* __restrict__ invdA, double* __restrict__ rhs,
                    double* __restrict__ x0, double* __restrict__ r0) {
  mom_side_rows<kTrac>(L, L.n, dir_index, dt, dtnu, W, R, p, udir, ndir, tn, A, invdA, rhs, x0,
                       r0, blockIdx.x, gridDim.x);
}

// The rows of the lattice's interior and coarse-edge nodes, [A.row0, A.n),
// one thread per row (momlat.hpp).
// A block's rows hold at most 7 entries each (checked at set-up), so its
// contiguous range of matrix values is staged in LDS and written out with
// consecutive lanes on consecutive values.
// Blocks [0, nbv) take the rows of the coarse vertices [0, A.row0) side-based
// (one group of kBlock / kRowLanes rows each), the others the lattice rows,
// so that the two kinds of work overlap.
template <bool kTrac>
__global__ void __launch_bounds__(kBlock) k_momentum_lat(DLevel L, MomLatArgs A, int nbv) {
  if ((int)blockIdx.x < nbv) {
    mom_side_rows<kTrac>(L, A.row0, A.dir_index, A.dt, A.dtnu, A.W, A.R, A.p, A.udir, A.ndir,
                         A.tn, A.A, A.invdA, A.rhs, A.x0, A.r0, blockIdx.x, nbv);
    return;
  }
  constexpr int kMaxVals = kBlock * 7;
  __shared__ double sa[kMaxVals];
  const int32_t r0 = A.row0 + (blockIdx.x - nbv) * kBlock;
  const int32_t r1 = r0 + kBlock < A.n ? r0 + kBlock : A.n;
  const int32_t base = A.rowptr[r0], top = A.rowptr[r1];
  const int32_t i = r0 + threadIdx.x;
  if (i < r1) mom_row<kTrac>(A, i, [&](int32_t s, double v) { sa[s - base] = v; });
  __syncthreads();
  for (int32_t q = threadIdx.x; q < top - base; q += kBlock) A.A[base + q] = sa[q];
}

// ------------------------------------------------------------------ BiCGSTAB
// Right-Jacobi-preconditioned BiCGSTAB on two right-hand sides sharing A.
// One iteration = five kernels:
//   B1  stopping test on r, rho = (r^, r), p = r + beta (p - omega v) (p = r in the
//       first iteration), p^ = D^-1 p
//   B2  v = A p^,                         partial (r^, v)
//   B3  alpha, s = r - alpha v (in r),    s^ = D^-1 s, partial (s, s)
//   B4  half-step test (x += alpha p^ and stop) or t = A s^, partials (t, s), (t, t)
//   B5  omega, x += alpha p^ + omega s^, r = s - omega t, partials (r, r), (r^, r)
// p^ and s^, the vectors the products gather, hold the two right-hand sides
// interleaved ([n][2]); the others hold them one after the other ([2][n]).

// The start: the assembly has written r = b - A x0 (x0 = W, the boundary
// values on Dirichlet rows); r^ = r, partial sums of (r, r) and (b, b).
__global__ void __launch_bounds__(kBlock)
k_bicg_start(int32_t n32, BicgVecs V, Scal* sc, double* part) {
  const int64_t n = n32;
  double rr[2] = {0, 0}, bb[2] = {0, 0};
  for (int64_t row = blockIdx.x * (int64_t)kBlock + threadIdx.x; row < n;
       row += (int64_t)gridDim.x * kBlock) {
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const double b = V.b[d * n + row];
      const double r = V.r[d * n + row];
      V.rhat[d * n + row] = r;
      rr[d] += r * r;
      bb[d] += b * b;
    }
  }
  const double vals[6] = {rr[0], rr[1], rr[0], rr[1], bb[0], bb[1]};
  const int idx[6] = {slot(SL_RR, 0), slot(SL_RR, 1), slot(SL_RHR, 0), slot(SL_RHR, 1),
                      slot(SL_BB, 0), slot(SL_BB, 1)};
  block_store<6>(vals, part, idx);
  if (blockIdx.x == 0 && threadIdx.x < 2) reset_scal(sc[threadIdx.x]);
}

__global__ void __launch_bounds__(kBlock)
k_bicg_b1(int32_t n32, BicgVecs V, Scal* sc, const double* part, int nb, int it, double tol,
          int my_stamp, int check_only) {
  const int64_t n = n32;
  bool act[2] = {active(sc, 0, my_stamp), active(sc, 1, my_stamp)};
  if (!act[0] && !act[1]) return;
  const int idx[6] = {slot(SL_RR, 0), slot(SL_RR, 1), slot(SL_RHR, 0), slot(SL_RHR, 1),
                      slot(SL_BB, 0), slot(SL_BB, 1)};
  double s6[6];
  block_sums<6>(part, nb, idx, s6);
  bool zero_rhs[2] = {false, false}, upd[2] = {false, false};
  double beta[2] = {0, 0}, omega[2] = {1, 1};
  for (int d = 0; d < 2; ++d) {
    if (!act[d]) continue;
    const double bb = it == 1 ? s6[4 + d] : sc[d].bb;
    const double rel = bb > 0.0 ? sqrt(s6[d] / bb) : 0.0;
    const bool nan = !isfinite(bb) || !isfinite(s6[d]) || !isfinite(rel);
    const bool fin = bb == 0.0 || nan || rel <= tol;
    zero_rhs[d] = bb == 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (it == 1) sc[d].bb = bb;
      sc[d].rel = rel;
      if (fin) {
        sc[d].done_stamp = my_stamp;
        sc[d].iters = it - 1;
        sc[d].status = nan ? 2 : 0;
      } else if (!check_only) {
        sc[d].rho[0] = s6[2 + d];
      }
    }
    if (!fin && !check_only) {
      upd[d] = true;
      beta[d] = (s6[2 + d] / sc[d].rho_old) * (sc[d].alpha / sc[d].omega);
      omega[d] = sc[d].omega;
    }
  }
  if (!upd[0] && !upd[1] && !zero_rhs[0] && !zero_rhs[1]) return;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double dinv = V.invd[i];
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      if (zero_rhs[d]) V.x[d * n + i] = 0.0;
      if (!upd[d]) continue;
      // the first direction is the residual itself (p and v are not read)
      const double pv = it == 1 ? V.r[d * n + i]
                                : V.r[d * n + i] + beta[d] * (V.p[d * n + i] - omega[d] * V.v[d * n + i]);
      V.p[d * n + i] = pv;
      V.phat[2 * i + d] = dinv * pv;
    }
  }
}

__global__ void __launch_bounds__(kBlock)
k_bicg_b2(DLevel L, const double* __restrict__ A, BicgVecs V, Scal* sc, double* part,
          int my_stamp) {
  if (!active(sc, 0, my_stamp) && !active(sc, 1, my_stamp)) return;
  __shared__ TileStage<double> st;
  const int64_t n = L.n;
  double dot[2] = {0, 0};
  for (int t = blockIdx.x; t < L.ntiles; t += gridDim.x) {
    const int r0 = L.tile[t], r1 = L.tile[t + 1];
    const int s0 = stage_tile<double, true>(st, L, A, r0, r1);
    const int row = r0 + threadIdx.x;
    if (row < r1) {
      double av[2];
      tile_row2(st, L, s0, row, reinterpret_cast<const double2*>(V.phat), av);
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        V.v[d * n + row] = av[d];
        dot[d] += V.rhat[d * n + row] * av[d];
      }
    }
  }
  const int idx[2] = {slot(SL_RHV, 0), slot(SL_RHV, 1)};
  block_store<2>(dot, part, idx);
}

__global__ void __launch_bounds__(kBlock)
k_bicg_b3(int32_t n32, BicgVecs V, Scal* sc, double* part, int nb, int my_stamp) {
  const int64_t n = n32;
  bool act[2] = {active(sc, 0, my_stamp), active(sc, 1, my_stamp)};
  if (!act[0] && !act[1]) return;
  const int idx[2] = {slot(SL_RHV, 0), slot(SL_RHV, 1)};
  double rhv[2];
  block_sums<2>(part, nb, idx, rhv);
  double alpha[2];
  for (int d = 0; d < 2; ++d) {
    alpha[d] = act[d] ? sc[d].rho[0] / rhv[d] : 0.0;
    if (act[d] && blockIdx.x == 0 && threadIdx.x == 0) sc[d].alpha = alpha[d];
  }
  double ss[2] = {0, 0};
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double dinv = V.invd[i];
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      if (!act[d]) continue;
      const double s = V.r[d * n + i] - alpha[d] * V.v[d * n + i];
      V.r[d * n + i] = s;
      V.shat[2 * i + d] = dinv * s;
      ss[d] += s * s;
    }
  }
  const int o[2] = {slot(SL_SS, 0), slot(SL_SS, 1)};
  block_store<2>(ss, part, o);
}

__global__ void __launch_bounds__(kBlock)
k_bicg_b4(DLevel L, const double* __restrict__ A, BicgVecs V, Scal* sc, double* part, int nb,
          int it, double tol, int my_stamp) {
  const int64_t n = L.n;
  bool act[2] = {active(sc, 0, my_stamp), active(sc, 1, my_stamp)};
  if (!act[0] && !act[1]) return;
  __shared__ TileStage<double> st;
  const int idx[2] = {slot(SL_SS, 0), slot(SL_SS, 1)};
  double ss[2];
  block_sums<2>(part, nb, idx, ss);
  bool half[2] = {false, false}, need_t = false;
  double alpha[2] = {0, 0};
  for (int d = 0; d < 2; ++d) {
    if (!act[d]) continue;
    const double rel = sqrt(ss[d] / sc[d].bb);
    const bool nan = !isfinite(rel);
    if (nan || rel <= tol) {
      half[d] = true;
      alpha[d] = sc[d].alpha;
      if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[d].rel = rel;
        sc[d].done_stamp = my_stamp;
        sc[d].iters = it;
        sc[d].status = nan ? 2 : 0;
      }
    } else {
      need_t = true;
    }
  }
  if (half[0] || half[1]) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
#pragma unroll
      for (int d = 0; d < 2; ++d)
        if (half[d]) V.x[d * n + i] += alpha[d] * V.phat[2 * i + d];
    }
  }
  if (!need_t) return;
  double ts[2] = {0, 0}, tt[2] = {0, 0};
  for (int t = blockIdx.x; t < L.ntiles; t += gridDim.x) {
    const int r0 = L.tile[t], r1 = L.tile[t + 1];
    const int s0 = stage_tile<double, true>(st, L, A, r0, r1);
    const int row = r0 + threadIdx.x;
    if (row < r1) {
      double at[2];
      tile_row2(st, L, s0, row, reinterpret_cast<const double2*>(V.shat), at);
#pragma unroll
      for (int d = 0; d < 2; ++d) {
        V.t[d * n + row] = at[d];
        ts[d] += at[d] * V.r[d * n + row];
        tt[d] += at[d] * at[d];
      }
    }
  }
  const double vals[4] = {ts[0], ts[1], tt[0], tt[1]};
  const int o[4] = {slot(SL_TS, 0), slot(SL_TS, 1), slot(SL_TT, 0), slot(SL_TT, 1)};
  block_store<4>(vals, part, o);
}

__global__ void __launch_bounds__(kBlock)
k_bicg_b5(int32_t n32, BicgVecs V, Scal* sc, double* part, int nb, int my_stamp) {
  const int64_t n = n32;
  bool act[2] = {active(sc, 0, my_stamp), active(sc, 1, my_stamp)};
  if (!act[0] && !act[1]) return;
  const int idx[4] = {slot(SL_TS, 0), slot(SL_TS, 1), slot(SL_TT, 0), slot(SL_TT, 1)};
  double s4[4];
  block_sums<4>(part, nb, idx, s4);
  double alpha[2] = {0, 0}, omega[2] = {0, 0};
  for (int d = 0; d < 2; ++d) {
    if (!act[d]) continue;
    alpha[d] = sc[d].alpha;
    omega[d] = s4[d] / s4[2 + d];
  }
  double rr[2] = {0, 0}, rhr[2] = {0, 0};
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      if (!act[d]) continue;
      const int64_t k = d * n + i;
      V.x[k] += alpha[d] * V.phat[2 * i + d] + omega[d] * V.shat[2 * i + d];
      const double r = V.r[k] - omega[d] * V.t[k];
      V.r[k] = r;
      rr[d] += r * r;
      rhr[d] += V.rhat[k] * r;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    for (int d = 0; d < 2; ++d)
      if (act[d]) {
        sc[d].omega = omega[d];
        sc[d].rho_old = sc[d].rho[0];
      }
  }
  const double vals[4] = {rr[0], rr[1], rhr[0], rhr[1]};
  const int o[4] = {slot(SL_RR, 0), slot(SL_RR, 1), slot(SL_RHR, 0), slot(SL_RHR, 1)};
  block_store<4>(vals, part, o);
}

// ------------------------------------------------------------------ PCG
// Jacobi-preconditioned CG (vectors of type T, dot products in FP64) in the
// single-reduction form of Chronopoulos and Gear (1989).  With z = D^-1 r,
// w = A z, gamma = (r, z), delta = (z, w):
//   beta_i  = gamma_i / gamma_{i-1},
//   alpha_i = gamma_i / (delta_i - beta_i gamma_i / alpha_{i-1}),
//   p_i = z_i + beta_i p_{i-1},  s_i = w_i + beta_i s_{i-1}  (so s_i = A p_i),
//   x_{i+1} = x_i + alpha_i p_i,  r_{i+1} = r_i - alpha_i s_i.
// In exact arithmetic these are the textbook iterates (A-conjugacy gives
// (p_i, A p_i) = delta_i - beta_i gamma_i / alpha_{i-1}); both dot products of
// an iteration share one reduction, so an iteration is one kernel:
//   K(it)  sums the partials of iteration it-1 (gamma, delta, (r, r)), tests
//          ||r_{it-1}|| <= tol ||b|| (iters = it - 1), forms alpha, beta, updates
//          the row's p, s, x, r and computes w_it = A z_it with z_it formed on
//          the fly at the gathered columns from r, w, s of iteration it-1,
//          then the partials of iteration it.
// r, w and s are read at neighbouring rows, so they alternate between two
// buffers (K(it) reads [(it-1) & 1], writes [it & 1]); x and p are row-local;
// z is recomputed where needed.  gamma and alpha alternate in the scalars the
// same way (written by block 0, read by every block from the other slot), and
// so do the partial-sum slots (K(it) sums parity (it-1) & 1 while its blocks
// store parity it & 1).

// r_0 = b - A x_0 (x_0 = 0 when zero_x0)
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_pcg_residual(DLevel L, PcgVecs<T> V, int zero_x0) {
  __shared__ TileStage<T> st;
  for (int t = blockIdx.x; t < L.ntiles; t += gridDim.x) {
    const int r0 = L.tile[t], r1 = L.tile[t + 1];
    int s0 = 0;
    if (!zero_x0) s0 = stage_tile(st, L, V.val, r0, r1);
    const int row = r0 + threadIdx.x;
    if (row < r1) {
      T ax[1] = {T(0)};
      if (!zero_x0) tile_row<T, 1>(st, L, s0, row, [&](int, int c) { return V.x[c]; }, ax);
      if (zero_x0) V.x[row] = T(0);
      V.r[0][row] = V.b[row] - ax[0];
    }
  }
}

// z_0 = D^-1 r_0, w_0 = A z_0 (z_0 formed at the gathered columns), partials
// gamma_0, delta_0, (r_0, r_0), (b, b); resets the solver scalars
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_pcg_start(DLevel L, PcgVecs<T> V, Scal* sc, double* part) {
  __shared__ TileStage<T> st;
  const T* __restrict__ r = V.r[0];
  const T* __restrict__ dinv = V.invd;
  double g = 0.0, dl = 0.0, rr = 0.0, bb = 0.0;
  for (int t = blockIdx.x; t < L.ntiles; t += gridDim.x) {
    const int r0 = L.tile[t], r1 = L.tile[t + 1];
    const int s0 = stage_tile(st, L, V.val, r0, r1);
    const int row = r0 + threadIdx.x;
    if (row < r1) {
      T az[1];
      tile_row<T, 1>(st, L, s0, row, [&](int, int c) { return dinv[c] * r[c]; }, az);
      const T rv = r[row], z = dinv[row] * rv, bv = V.b[row];
      V.w[0][row] = az[0];
      g += (double)rv * (double)z;
      dl += (double)z * (double)az[0];
      rr += (double)rv * (double)rv;
      bb += (double)bv * (double)bv;
    }
  }
  const double vals[4] = {g, dl, rr, bb};
  const int idx[4] = {slot(SL_RZ, 0), slot(SL_PQ, 0), slot(SL_RR, 0), slot(SL_BB, 0)};
  block_store<4>(vals, part, idx);
  if (blockIdx.x == 0 && threadIdx.x == 0) reset_scal(sc[0]);
}

// One thread per row on the ELL copy, so a row's indices and values are one
// coalesced load away from the thread and the gathers follow directly.
template <typename T>
__global__ void __launch_bounds__(kBlock)
k_pcg_iter(int32_t n, PcgVecs<T> V, Scal* sc, double* part, int nb, int it, double tol,
           int my_stamp, int check_only) {
  const int po = (it - 1) & 1, pn = it & 1;
  // the solver scalars are read together with the first operands (reading
  // after the solve has finished is harmless; nothing is written until the
  // stamp has been tested)
  const int stamp0 = sc[0].done_stamp;
  const double bb_prev = sc[0].bb, gam_prev = sc[0].rho[pn], al_prev = sc[0].pcg_alpha[po];
  const T* __restrict__ ro = V.r[po];
  const T* __restrict__ wo = V.w[po];
  const T* __restrict__ so = V.s[po];
  const T* __restrict__ dinv = V.invd;
  const int32_t* __restrict__ ecol = V.ell_col;
  const T* __restrict__ eval = V.ell_val;
  const int w = V.ell_w;
  const int64_t ln = n;
  const bool start = it == 1;  // p_0 = z_0, s_0 = w_0
  T alpha = T(0), beta = T(0);
  double g = 0.0, dl = 0.0, rr = 0.0;
  const int first_row = blockIdx.x * kBlock + threadIdx.x;
  T xr = T(0), pr = T(0), rv = T(0), wv = T(0), sv = T(0), dv = T(0);
  T gv[kRowBatch], gr[kRowBatch], gw[kRowBatch], gs[kRowBatch];
  // Loads carry no per-entry conditions, so that all of a batch's index loads
  // are in flight together and then all of its gathers (a condition per entry
  // splits the batch into blocks that each wait for their own index).  The
  // ELL width is a multiple of kRowBatch; padding entries are (row, 0).  p and
  // s are read even at it = 1, where they are not used.
  auto load_row = [&](int row) {
    xr = V.x[row];
    rv = ro[row];
    wv = wo[row];
    dv = dinv[row];
    pr = V.p[row];
    sv = so[row];
  };
  auto load_batch = [&](int row, int k0) {
    int cix[kRowBatch];
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) {
      const int64_t e = (int64_t)(k0 + u) * ln + row;
      cix[u] = ecol[e];
      gv[u] = eval[e];
    }
#pragma unroll
    for (int u = 0; u < kRowBatch; ++u) {
      const int c = cix[u];
      gr[u] = ro[c];
      gw[u] = wo[c];
      gs[u] = so[c];
    }
  };
  // the first row's operands and gathers are issued before the reduction of
  // the partial sums (alpha and beta are needed only to combine them)
  if (first_row < n) {
    load_row(first_row);
    load_batch(first_row, 0);
  }
  if (!(stamp0 == 0 || stamp0 >= my_stamp)) return;  // solve already finished
  {
    const int idx[4] = {slot(SL_RZ, po), slot(SL_PQ, po), slot(SL_RR, po), slot(SL_BB, 0)};
    double sm[4];
    block_sums<4>(part, nb, idx, sm);
    const double bb = start ? sm[3] : bb_prev;
    const double rel = bb > 0.0 ? sqrt(sm[2] / bb) : 0.0;
    const bool nan = !isfinite(bb) || !isfinite(sm[2]) || !isfinite(rel);
    const bool fin = bb == 0.0 || nan || rel <= tol;
    double al = 0.0, be = 0.0;
    if (!fin) {
      be = start ? 0.0 : sm[0] / gam_prev;
      al = start ? sm[0] / sm[1] : sm[0] / (sm[1] - be * sm[0] / al_prev);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      if (start) sc[0].bb = bb;
      sc[0].rel = rel;
      if (fin) {
        sc[0].done_stamp = my_stamp;
        sc[0].iters = it - 1;
        sc[0].status = nan ? 2 : 0;
      } else {
        sc[0].rho[po] = sm[0];
        sc[0].pcg_alpha[pn] = al;
        sc[0].alpha = al;
      }
    }
    if (bb == 0.0) {  // zero right-hand side: the solution is zero
      for (int i = first_row; i < n; i += gridDim.x * kBlock) V.x[i] = T(0);
      return;
    }
    if (fin || check_only) return;
    alpha = (T)al;
    beta = (T)be;
  }
  for (int row = first_row; row < n; row += gridDim.x * kBlock) {
    if (row != first_row) {
      load_row(row);
      load_batch(row, 0);
    }
    const T zo = dv * rv;
    const T pnw = start ? zo : zo + beta * pr;
    const T sn = start ? wv : wv + beta * sv;
    const T rn = rv - alpha * sn;
    const T zn = dv * rn;
    // w_it at this row: z_it of each neighbour from its r, w, s of it-1, in
    // row order in batches of kRowBatch
    T acc = T(0);
    for (int k0 = 0; k0 < w; k0 += kRowBatch) {
      if (k0 > 0) load_batch(row, k0);
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) {
        const T snc = start ? gw[u] : gw[u] + beta * gs[u];
        acc += gv[u] * (gr[u] - alpha * snc);  // ELL values hold K_ij / K_jj
      }
    }
    V.x[row] = xr + alpha * pnw;
    V.p[row] = pnw;
    V.r[pn][row] = rn;
    V.s[pn][row] = sn;
    V.w[pn][row] = acc;
    g += (double)rn * (double)zn;
    dl += (double)zn * (double)acc;
    rr += (double)rn * (double)rn;
  }
  // this kernel reads the partials of it-1 while other blocks may already be
  // storing those of it: the two use the slots of opposite parity
  const double vals[3] = {g, dl, rr};
  const int o[3] = {slot(SL_RZ, pn), slot(SL_PQ, pn), slot(SL_RR, pn)};
  block_store<3>(vals, part, o);
}

// ELL copy of a CSR matrix (row order kept: diagonal first, then columns
// ascending; padding (i, 0))
// ELL copies of a CSR matrix K: column indices, K in FP64, and K D^-1 (each
// column scaled by 1 / K_jj, so that products with z = D^-1 r need no
// gather of the diagonal) in FP64 and FP32.
__global__ void k_make_ell(DLevel L, const double* __restrict__ val,
                           const double* __restrict__ invd, int w, int32_t* __restrict__ ecol,
                           double* __restrict__ ev, double* __restrict__ evs,
                           float* __restrict__ evs32) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < L.n; i += gridDim.x * blockDim.x) {
    const int beg = L.rowptr[i], len = L.rowptr[i + 1] - beg;
    for (int k = 0; k < w; ++k) {
      const int64_t e = (int64_t)k * L.n + i;
      const bool in = k < len;
      const int c = in ? L.col[beg + k] : i;
      const double v = in ? val[beg + k] : 0.0;
      const double vs = v * invd[c];
      ecol[e] = c;
      ev[e] = v;
      evs[e] = vs;
      evs32[e] = (float)vs;
    }
  }
}

// ------------------------------------------------------------------ restriction
// Coarse divergence tested with the coarse shape functions against the fine
// velocity: (Dbar U)_I = sum over fine triangles e of (int_e div u_h)
// * (mean of psi_I^c over e).  psi_I^c is linear on e, so its mean is the
// mean of its values at e's vertices, i.e. of their barycentric coordinates in
// the coarse ancestor T = e >> 2k.  Those follow from e's index: the children
// of triangle t are 4t..4t+3, so the base-4 digits of e below T are the child
// choices (0: corner a, 1: corner b, 2: corner c, 3: middle).  One thread per
// fine triangle; the 4^k triangles of T are consecutive lanes (4^k <= 64),
// reduced with a segmented butterfly into tripart[T][3].
__global__ void __launch_bounds__(kBlock)
k_restrict_galerkin(const int32_t* __restrict__ tri, int32_t nt, const double2* __restrict__ xy,
                    int levels, const double* __restrict__ ut, int64_t stride,
                    double* __restrict__ tripart) {
  const int seg = 1 << (2 * levels);
  const double wscale = 1.0 / (double)(3 << levels);
  for (int e0 = blockIdx.x * blockDim.x; e0 < nt; e0 += gridDim.x * blockDim.x) {
    const int e = e0 + threadIdx.x;
    double c[3] = {0.0, 0.0, 0.0};
    if (e < nt) {
      int B[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
      for (int l = levels - 1; l >= 0; --l) {
        const int ch = (e >> (2 * l)) & 3;
        int nbv[3][3];
        for (int w = 0; w < 3; ++w) {
          const int ab = B[0][w] + B[1][w], bc = B[1][w] + B[2][w], ca = B[2][w] + B[0][w];
          if (ch == 0) {
            nbv[0][w] = 2 * B[0][w]; nbv[1][w] = ab; nbv[2][w] = ca;
          } else if (ch == 1) {
            nbv[0][w] = ab; nbv[1][w] = 2 * B[1][w]; nbv[2][w] = bc;
          } else if (ch == 2) {
            nbv[0][w] = ca; nbv[1][w] = bc; nbv[2][w] = 2 * B[2][w];
          } else {
            nbv[0][w] = ab; nbv[1][w] = bc; nbv[2][w] = ca;
          }
        }
        for (int v = 0; v < 3; ++v)
          for (int w = 0; w < 3; ++w) B[v][w] = nbv[v][w];
      }
      const int v0 = tri[3 * e], v1 = tri[3 * e + 1], v2 = tri[3 * e + 2];
      const double2 p0 = xy[v0], p1 = xy[v1], p2 = xy[v2];
      const double b0 = p1.y - p2.y, c0 = p2.x - p1.x;
      const double b1 = p2.y - p0.y, c1 = p0.x - p2.x;
      const double b2 = p0.y - p1.y, c2 = p1.x - p0.x;
      // int_e div u_h = sum_j (b_j u_j + c_j v_j) / 2
      const double I = 0.5 * (b0 * ut[v0] + c0 * ut[stride + v0] + b1 * ut[v1] +
                              c1 * ut[stride + v1] + b2 * ut[v2] + c2 * ut[stride + v2]);
      for (int w = 0; w < 3; ++w) c[w] = I * (double)(B[0][w] + B[1][w] + B[2][w]) * wscale;
    }
    for (int o = seg >> 1; o > 0; o >>= 1)
      for (int w = 0; w < 3; ++w) c[w] += __shfl_xor(c[w], o, 64);
    if (e < nt && (e & (seg - 1)) == 0) {
      const int T = e >> (2 * levels);
      for (int w = 0; w < 3; ++w) tripart[3 * T + w] = c[w];
    }
  }
}

__global__ void __launch_bounds__(kBlock)
k_restrict_nodes(int32_t nc, const int32_t* __restrict__ cn_ptr, const int32_t* __restrict__ cn_tri,
                 const double* __restrict__ tripart, const uint8_t* __restrict__ nat, double scale,
                 double* __restrict__ b, double* part) {
  double sum = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += gridDim.x * blockDim.x) {
    double dv = 0.0;
    for (int q = cn_ptr[i]; q < cn_ptr[i + 1]; ++q) {
      const int e = cn_tri[q];
      dv += tripart[3 * (e >> 2) + (e & 3)];
    }
    const double v = nat[i] ? 0.0 : scale * dv;
    b[i] = v;
    sum += v;
  }
  const double vals[1] = {sum};
  const int idx[1] = {0};
  block_store<1>(vals, part, idx);
}

__global__ void __launch_bounds__(kBlock)
k_restrict_inject(DLevel C, const uint8_t* __restrict__ nat, const double* __restrict__ ut,
                  int64_t stride, double scale, double* __restrict__ b, double* part) {
  double sum = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < C.n; i += gridDim.x * blockDim.x) {
    const int beg = C.rowptr[i], end = C.rowptr[i + 1];
    const double2 pi = C.xy[i];
    const double ui = ut[i], vi = ut[stride + i];
    double dv = 0.0;
    for (int s = beg + 1; s < end; ++s) {
      const int j = C.col[s];
      const double2 pj = C.xy[j];
      const double uj = ut[j], vj = ut[stride + j];
      for (int q = 0; q < 2; ++q) {
        const int k = C.side[2 * s + q];
        if (k < 0) continue;
        const SideGeo g = side_geo(pi, pj, C.xy[k], q == 0 ? 1.0 : -1.0);
        dv += (g.bj * uj + g.cj * vj) * (1.0 / 6.0) + (g.bi * ui + g.ci * vi) * (1.0 / 12.0);
      }
    }
    const double v = nat[i] ? 0.0 : scale * dv;
    b[i] = v;
    sum += v;
  }
  const double vals[1] = {sum};
  const int idx[1] = {0};
  block_store<1>(vals, part, idx);
}

// v -= sum(part slot 0) / n, or with weights: v -= (sum w v) / (sum w) where
// part slot 0 holds sum w v and slot 1 sum w.
__global__ void __launch_bounds__(kBlock)
k_remove_mean(int32_t n, double* __restrict__ v, const double* part, int nb, int weighted) {
  const int idx[2] = {0, kNbMax};
  double s[2];
  block_sums<2>(part, nb, idx, s);
  const double mean = weighted ? s[0] / s[1] : s[0] / (double)n;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    v[i] -= mean;
}

__global__ void __launch_bounds__(kBlock)
k_weighted_sums(int32_t n, const double* __restrict__ v, const double* __restrict__ w,
                double* part) {
  double a = 0.0, b = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    a += w[i] * v[i];
    b += w[i];
  }
  const double vals[2] = {a, b};
  const int idx[2] = {0, kNbMax};
  block_store<2>(vals, part, idx);
}

// ------------------------------------------------------------------ prolongation
// Every fine node is the coarse P1 function evaluated there: with the coarse
// triangle T holding the node and its barycentric coordinates n/2^k,
// phi_f = (n0 phi[T0] + n1 phi[T1] + n2 phi[T2]) / 2^k (dyadic weights, exact).
__global__ void __launch_bounds__(kBlock)
k_prolong(int32_t nf, const int32_t* __restrict__ pcode, const int32_t* __restrict__ tri_c,
          int levels, const double* __restrict__ phic, double* __restrict__ phif) {
  const int den = 1 << levels;
  const double inv = 1.0 / (double)den;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < nf; i += gridDim.x * blockDim.x) {
    const int2 code = reinterpret_cast<const int2*>(pcode)[i];
    const int T = code.x;
    const int n1 = code.y & 0xffff, n2 = code.y >> 16, n0 = den - n1 - n2;
    const double f = (double)n0 * phic[tri_c[3 * T]] + (double)n1 * phic[tri_c[3 * T + 1]] +
                     (double)n2 * phic[tri_c[3 * T + 2]];
    phif[i] = f * inv;
  }
}


// ------------------------------------------------------------------ correction
// Right-hand sides of Eqs. 25-26: -(2/3) dt G phi_f on non-Dirichlet rows (0
// on Dirichlet rows) and -nu D U~; one lane group per row.
// MODE CGP_MASS_CONSISTENT: the right-hand sides of the velocity correction
// (2, Dirichlet rows 0) and, for chi = 1, of the rotational pressure update
// (3rd), interleaved per node for the fused Chebyshev solve.
// MODE CGP_MASS_LUMPED_P (chi = 1): the velocity right-hand sides as above,
// and the pressure update of Eq. 27 written directly, p_out = p_in + phi +
// (-nu D U~)_i / m_i with the lumped mass m_i = 2 M_ii (the P1 row sum).
// MODE CGP_MASS_LUMPED: U and P written directly, dU = rhs / m_i.
__global__ void __launch_bounds__(kBlock)
k_correct_rhs(DLevel L, const int32_t* __restrict__ dir_index, const double* __restrict__ M,
              double dt, double nu, int chi, int mode, const double* __restrict__ phi,
              const double* __restrict__ ut, const double* __restrict__ p_in,
              double* __restrict__ rhs, double* __restrict__ u_out, double* __restrict__ p_out,
              const int32_t* __restrict__ lat_of) {
  const int64_t n = L.n;
  const int lane = threadIdx.x % kRowLanes, rpb = kBlock / kRowLanes;
  for (int base = blockIdx.x * rpb; base < n; base += gridDim.x * rpb) {
    const int i = base + threadIdx.x / kRowLanes;
    if (i >= n) continue;  // uniform within the lane group
    const int beg = L.rowptr[i], end = L.rowptr[i + 1];
    const double2 pi = L.xy[i];
    const double phii = phi[i];
    const double ui = ut[i], vi = ut[n + i];
    double acc[3] = {0.0, 0.0, 0.0};  // gx, gy, div
    // as in the momentum assembly: every gather of a lane's two slots is
    // issued before any arithmetic (a missing side reads node j instead)
    struct Slot {
      int2 sd;
      double2 pj, pk[2];
      double phj, uj, vj;
    };
    const int2* side2 = reinterpret_cast<const int2*>(L.side);
    auto load = [&](int s, Slot& d) {
      const int j = L.col[s];
      d.sd = side2[s];
      const int k0 = d.sd.x >= 0 ? d.sd.x : j, k1 = d.sd.y >= 0 ? d.sd.y : j;
      d.pj = L.xy[j];
      d.phj = phi[j];
      d.uj = chi ? ut[j] : 0.0;
      d.vj = chi ? ut[n + j] : 0.0;
      d.pk[0] = L.xy[k0];
      d.pk[1] = L.xy[k1];
    };
    auto add = [&](const Slot& d) {
      const double ph = d.phj + 0.5 * phii;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        if ((q == 0 ? d.sd.x : d.sd.y) < 0) continue;
        const SideGeo g = side_geo(pi, d.pj, d.pk[q], q == 0 ? 1.0 : -1.0);
        acc[0] += g.bi * ph;
        acc[1] += g.ci * ph;
        if (chi)
          acc[2] += (g.bj * d.uj + g.cj * d.vj) * (1.0 / 6.0) + (g.bi * ui + g.ci * vi) * (1.0 / 12.0);
      }
    };
    for (int s0 = beg + 1 + lane; s0 < end; s0 += 2 * kRowLanes) {
      const int s1 = s0 + kRowLanes;
      const bool two = s1 < end;
      Slot a, b;
      load(s0, a);
      load(two ? s1 : s0, b);
      add(a);
      if (two) add(b);
    }
    group_sum<3>(acc);
    if (lane == 0) {
      const bool dir = dir_index[i] >= 0;
      const double rx = dir ? 0.0 : (dt / 9.0) * acc[0];
      const double ry = dir ? 0.0 : (dt / 9.0) * acc[1];
      const double rp = -nu * acc[2];
      // mass-solve right-hand sides go to the lattice layout
      const int64_t li = lat_of[i];
      if (mode == CGP_MASS_CONSISTENT) {
        const int nr = chi ? 3 : 2;
        rhs[li * nr] = rx;
        rhs[li * nr + 1] = ry;
        if (chi) rhs[li * nr + 2] = rp;
      } else {
        const double ml = 2.0 * M[beg];  // lumped mass: row sum of M
        if (mode == CGP_MASS_LUMPED_P) {
          rhs[li * 2] = rx;
          rhs[li * 2 + 1] = ry;
        } else {
          u_out[i] = ui + rx / ml;
          u_out[n + i] = vi + ry / ml;
        }
        // p_in == nullptr: the increment is the pressure (non-incremental)
        const double pold = p_in ? p_in[i] : 0.0;
        p_out[i] = chi ? pold + phii + rp / ml : pold + phii;
      }
    }
  }
}

// u_out = U~ + dU, p_out = p_in + phi_f (+ dp) unless write_p is 0; du holds
// (dU_x, dU_y[, dp]) interleaved per node
__global__ void __launch_bounds__(kBlock)
k_final_update(int32_t n32, const double* __restrict__ ut, const double* __restrict__ du,
               const double* p_in, const double* __restrict__ phi, int nr, int write_p,
               double* __restrict__ u_out, double* p_out, const int32_t* __restrict__ lat_of) {
  const int64_t n = n32;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int64_t k = (int64_t)lat_of[i] * nr;
    u_out[i] = ut[i] + du[k];
    u_out[n + i] = ut[n + i] + du[k + 1];
    if (write_p) {
      const double pv = (p_in ? p_in[i] : 0.0) + phi[i];  // p_in == nullptr: P = phi
      p_out[i] = nr == 3 ? pv + du[k + 2] : pv;
    }
  }
}

// The same with dU (and dp) as the sum of the two float solves of the
// mixed-precision mass solves, added in FP64.
__global__ void __launch_bounds__(kBlock)
k_final_update2(int32_t n32, const double* __restrict__ ut, const float* __restrict__ d1,
                const float* __restrict__ d2, const double* p_in, const double* __restrict__ phi,
                int nr, int write_p, double* __restrict__ u_out, double* p_out,
                const int32_t* __restrict__ lat_of) {
  const int64_t n = n32;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int64_t k = (int64_t)lat_of[i] * nr;
    u_out[i] = ut[i] + ((double)d1[k] + (double)d2[k]);
    u_out[n + i] = ut[n + i] + ((double)d1[k + 1] + (double)d2[k + 1]);
    if (write_p) {
      const double pv = (p_in ? p_in[i] : 0.0) + phi[i];  // p_in == nullptr: P = phi
      p_out[i] = nr == 3 ? pv + ((double)d1[k + 2] + (double)d2[k + 2]) : pv;
    }
  }
}

// ------------------------------------------------------------------ guess guard
// Partial sums of ||b - K x||^2 for two candidate initial guesses (FP64).
__global__ void __launch_bounds__(kBlock)
k_guard_residuals(DLevel C, const double* __restrict__ K, const double* __restrict__ b,
                  const double* __restrict__ x0, const double* __restrict__ x1, double* part) {
  __shared__ TileStage<double> st;
  double rr[2] = {0.0, 0.0};
  for (int t = blockIdx.x; t < C.ntiles; t += gridDim.x) {
    const int r0 = C.tile[t], r1 = C.tile[t + 1];
    const int s0 = stage_tile(st, C, K, r0, r1);
    const int row = r0 + threadIdx.x;
    if (row < r1) {
      double kx[2];
      tile_row<double, 2>(st, C, s0, row, [&](int d, int c) { return d ? x1[c] : x0[c]; }, kx);
      const double bv = b[row];
#pragma unroll
      for (int d = 0; d < 2; ++d) rr[d] += (bv - kx[d]) * (bv - kx[d]);
    }
  }
  const int idx[2] = {slot(SL_RR, 0), slot(SL_RR, 1)};
  block_store<2>(rr, part, idx);
}

// Copies the candidate with the smaller residual (x0 on ties) into out.
__global__ void __launch_bounds__(kBlock)
k_guard_select(int32_t n, const double* __restrict__ x0, const double* __restrict__ x1,
               double* __restrict__ out, int32_t* chose, const double* part, int nb) {
  const int idx[2] = {slot(SL_RR, 0), slot(SL_RR, 1)};
  double s[2];
  block_sums<2>(part, nb, idx, s);
  const bool first = s[0] <= s[1] && isfinite(s[0]);
  if (blockIdx.x == 0 && threadIdx.x == 0) *chose = first ? 0 : 1;
  const double* src = first ? x0 : x1;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    out[i] = src[i];
}

// ------------------------------------------------------------------ small ops
// Copies n solver-scalar records into host-mapped pinned memory (the host
// polls them after an event): one 8-byte word per lane, then a system-scope
// fence.  Much cheaper on the stream than a DMA/blit copy of 72 bytes.
__global__ void k_mirror(const Scal* __restrict__ src, Scal* dst, int n) {
  constexpr int kWords = sizeof(Scal) / 8;
  static_assert(sizeof(Scal) % 8 == 0, "Scal is a whole number of words");
  const int i = threadIdx.x;
  if (i < n * kWords) {
    const int64_t* s = reinterpret_cast<const int64_t*>(src);
    int64_t* d = reinterpret_cast<int64_t*>(dst);
    d[i] = s[i];
  }
  __threadfence_system();
}

__global__ void k_copy(const double* __restrict__ a, double* __restrict__ b, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    b[i] = a[i];
}
__global__ void k_zero_masked(double* __restrict__ x, const uint8_t* __restrict__ nat, int32_t n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    if (nat[i]) x[i] = 0.0;
}
// x += d (FP32 correction into the FP64 iterate); returns at once when
// `skip` is given and its solve is done
__global__ void k_axpy_f32(const float* __restrict__ d, double* __restrict__ x, int64_t n,
                           const Scal* skip) {
  if (skip && skip->done_stamp) return;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] += (double)d[i];
}

__global__ void k_fill32(float* __restrict__ x, float v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

// r = b - K x in FP64 (and its FP32 copy), partials (r, r) and (b, b)
__global__ void __launch_bounds__(kBlock)
k_residual64(DLevel C, const double* __restrict__ K, const double* __restrict__ b,
             const double* __restrict__ x, double* __restrict__ r, float* __restrict__ r32,
             double* part) {
  __shared__ TileStage<double> st;
  double rr = 0.0, bb = 0.0;
  for (int t = blockIdx.x; t < C.ntiles; t += gridDim.x) {
    const int r0 = C.tile[t], r1 = C.tile[t + 1];
    const int s0 = stage_tile(st, C, K, r0, r1);
    const int row = r0 + threadIdx.x;
    if (row < r1) {
      double ax[1];
      tile_row<double, 1>(st, C, s0, row, [&](int, int c) { return x[c]; }, ax);
      const double bv = b[row];
      const double rv = bv - ax[0];
      r[row] = rv;
      r32[row] = (float)rv;
      rr += rv * rv;
      bb += bv * bv;
    }
  }
  const double vals[2] = {rr, bb};
  const int idx[2] = {slot(SL_RR, 0), slot(SL_BB, 0)};
  block_store<2>(vals, part, idx);
}

// one block: relative residual of the outer refinement loop into sc[0]
__global__ void k_reduce_check(const double* part, int nb, double tol, Scal* sc, int outer) {
  const int idx[2] = {slot(SL_RR, 0), slot(SL_BB, 0)};
  double s[2];
  block_sums<2>(part, nb, idx, s);
  if (threadIdx.x == 0) {
    const double rel = s[1] > 0.0 ? sqrt(s[0] / s[1]) : 0.0;
    const bool nan = !isfinite(s[0]) || !isfinite(s[1]) || !isfinite(rel);
    sc[0].bb = s[1];
    sc[0].rel = rel;
    sc[0].status = nan ? 2 : 0;
    sc[0].done_stamp = (nan || rel <= tol || s[1] == 0.0) ? outer + 1 : 0;
  }
}

// ------------------------------------------------ PCG with a factor preconditioner
// Textbook PCG (two reductions per iteration) around z = M^-1 r from the
// nested-dissection factor: partials of (r, z); the new direction with
// q = K p (p formed on the fly at the gathered columns, so p alternates
// between two buffers); the update of x and r.  rho of even / odd
// iterations alternates in the scalars as in the single-reduction PCG.

__global__ void __launch_bounds__(kBlock)
k_fpcg_rz(int32_t n, const double* __restrict__ r, const double* __restrict__ z, double* part,
          const Scal* skip) {
  if (skip && skip->done_stamp) return;
  double t = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) t += r[i] * z[i];
  const double vals[1] = {t};
  const int o[1] = {slot(SL_RZ, 0)};
  block_store<1>(vals, part, o);
}

__global__ void __launch_bounds__(kBlock)
k_fpcg_dir(int32_t n, const int32_t* __restrict__ ecol, const double* __restrict__ eval, int ew,
           const double* __restrict__ z, const double* __restrict__ pold, double* __restrict__ pnew,
           double* __restrict__ q, Scal* sc, double* part, int nb, int it, const Scal* skip) {
  if (skip && skip->done_stamp) return;
  const int idx[1] = {slot(SL_RZ, 0)};
  double rz[1];
  block_sums<1>(part, nb, idx, rz);
  const double rho_prev = sc[0].rho[(it - 1) & 1];
  const bool first = it == 1;
  const double beta = first || rho_prev == 0.0 ? 0.0 : rz[0] / rho_prev;
  if (blockIdx.x == 0 && threadIdx.x == 0) sc[0].rho[it & 1] = rz[0];
  const int64_t ln = n;
  double pq = 0.0;
  for (int row = blockIdx.x * kBlock + threadIdx.x; row < n; row += gridDim.x * kBlock) {
    const double pr = first ? z[row] : z[row] + beta * pold[row];
    double acc = 0.0;
    for (int k0 = 0; k0 < ew; k0 += kRowBatch) {
      int cix[kRowBatch];
      double gv[kRowBatch], gz[kRowBatch], gp[kRowBatch];
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) {
        const int64_t e = (int64_t)(k0 + u) * ln + row;
        cix[u] = ecol[e];
        gv[u] = eval[e];
      }
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) {
        gz[u] = z[cix[u]];
        gp[u] = first ? 0.0 : pold[cix[u]];
      }
#pragma unroll
      for (int u = 0; u < kRowBatch; ++u) acc += gv[u] * (gz[u] + beta * gp[u]);
    }
    pnew[row] = pr;
    q[row] = acc;
    pq += pr * acc;
  }
  const double vals[1] = {pq};
  const int o[1] = {slot(SL_PQ, 0)};
  block_store<1>(vals, part, o);
}

__global__ void __launch_bounds__(kBlock)
k_fpcg_update(int32_t n, const double* __restrict__ p, const double* __restrict__ q,
              double* __restrict__ x, double* __restrict__ r, const Scal* sc, double* part, int nb,
              int it, const Scal* skip) {
  if (skip && skip->done_stamp) return;
  const int idx[1] = {slot(SL_PQ, 0)};
  double pq[1];
  block_sums<1>(part, nb, idx, pq);
  const double rho = sc[0].rho[it & 1];
  const double alpha = pq[0] != 0.0 ? rho / pq[0] : 0.0;
  double rr = 0.0;
  for (int i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    x[i] += alpha * p[i];
    const double rn = r[i] - alpha * q[i];
    r[i] = rn;
    rr += rn * rn;
  }
  const double vals[1] = {rr};
  const int o[1] = {slot(SL_RR, 0)};
  block_store<1>(vals, part, o);
}

__global__ void k_fill(double* __restrict__ x, double v, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    x[i] = v;
}

inline int grid_for(int64_t units, int per_block, int cap = 4096) {
  int64_t g = (units + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

inline int row_group_grid(int64_t rows) { return grid_for(rows, kBlock / kRowLanes, 8192); }

}  // namespace

// ------------------------------------------------------------------ launchers

void launch_mass_assemble(const DLevel& L, double* Mval, hipStream_t s) {
  k_mass_assemble<<<grid_for(L.n, kBlock), kBlock, 0, s>>>(L, Mval);
}

namespace {
// vval[k] = Mval[vpos[k]] (0 where vpos is -1): the coarse-vertex rows of the
// lattice mass operator from the assembled CSR values
__global__ void k_vertex_rows(int64_t n, const int32_t* __restrict__ vpos,
                              const double* __restrict__ Mval, double* __restrict__ vval) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) vval[i] = vpos[i] >= 0 ? Mval[vpos[i]] : 0.0;
}
}  // namespace

void launch_vertex_rows(int64_t n, const int32_t* vpos, const double* Mval, double* vval,
                        hipStream_t s) {
  if (n > 0) k_vertex_rows<<<grid_for(n, kBlock), kBlock, 0, s>>>(n, vpos, Mval, vval);
}

void launch_coarse_assemble(const DLevel& L, const uint8_t* nat, double* Kval, float* Kval32,
                            double* Dxval, double* Dyval, double* invd, float* invd32,
                            double* lumped, hipStream_t s) {
  k_coarse_assemble<<<grid_for(L.n, kBlock), kBlock, 0, s>>>(L, nat, Kval, Kval32, Dxval, Dyval,
                                                             invd, invd32, lumped);
}

void launch_momentum_assemble(const DLevel& L, const int32_t* dir_index, double dt, double nu,
                              const double* u_prev, const double* u, const double* p,
                              const double* u_dir, int32_t n_dir, const double* f,
                              const double* t_nat, double* Aval, double* invdA, double* rhs,
                              double* x0, double* r0, double* scratch_w, double* scratch_r,
                              hipStream_t s, hipEvent_t* ev, const MomLattice* ml) {
  double2* W = reinterpret_cast<double2*>(scratch_w);
  double2* R = reinterpret_cast<double2*>(scratch_r);
  if (ev) (void)hipEventRecord(ev[0], s);
  k_momentum_fields<<<grid_for(L.n, kBlock), kBlock, 0, s>>>(L.n, u_prev, u, f, dt, W, R);
  if (!ml || ml->row0 >= L.n) {  // every row side-based
    if (t_nat)
      k_momentum_assemble<true><<<row_group_grid(L.n), kBlock, 0, s>>>(
          L, dir_index, dt, dt * nu, W, R, p, u_dir, n_dir, t_nat, Aval, invdA, rhs, x0, r0);
    else
      k_momentum_assemble<false><<<row_group_grid(L.n), kBlock, 0, s>>>(
          L, dir_index, dt, dt * nu, W, R, p, u_dir, n_dir, nullptr, Aval, invdA, rhs, x0, r0);
  } else {
    // the coarse-vertex rows [0, row0) side-based, the rest on the lattice,
    // in one launch
    const int32_t row0 = ml->row0;
    const MomLatArgs A{L.n, row0, L.rowptr, ml->slot, ml->rows, ml->tris, dir_index, W, R,
                       p,   u_dir, n_dir,   t_nat,    dt,       dt * nu,  Aval,      invdA,
                       rhs, x0,    r0};
    const int nbv = (row0 + kBlock / kRowLanes - 1) / (kBlock / kRowLanes);
    const int g = nbv + (int)((L.n - row0 + kBlock - 1) / kBlock);
    if (t_nat)
      k_momentum_lat<true><<<g, kBlock, 0, s>>>(L, A, nbv);
    else
      k_momentum_lat<false><<<g, kBlock, 0, s>>>(L, A, nbv);
  }
  if (ev) (void)hipEventRecord(ev[1], s);
}

void launch_bicg_start(int32_t n, const BicgVecs& V, Scal* sc, double* part, int nb,
                       hipStream_t s) {
  k_bicg_start<<<nb, kBlock, 0, s>>>(n, V, sc, part);
}

void launch_bicg_iter(const DLevel& L, const double* Aval, const BicgVecs& V, Scal* sc,
                      double* part, int nb, int it, double tol, bool check_only,
                      hipStream_t s, hipEvent_t* ev) {
  k_bicg_b1<<<nb, kBlock, 0, s>>>(L.n, V, sc, part, nb, it, tol, stamp(it, 1), check_only ? 1 : 0);
  if (check_only) return;
  if (ev) (void)hipEventRecord(ev[0], s);
  k_bicg_b2<<<nb, kBlock, 0, s>>>(L, Aval, V, sc, part, stamp(it, 2));
  if (ev) (void)hipEventRecord(ev[1], s);
  k_bicg_b3<<<nb, kBlock, 0, s>>>(L.n, V, sc, part, nb, stamp(it, 3));
  k_bicg_b4<<<nb, kBlock, 0, s>>>(L, Aval, V, sc, part, nb, it, tol, stamp(it, 4));
  k_bicg_b5<<<nb, kBlock, 0, s>>>(L.n, V, sc, part, nb, stamp(it, 5));
}

template <typename T>
void launch_pcg_init(const DLevel& L, const PcgVecs<T>& V, bool zero_x0, Scal* sc, double* part,
                     int nb, hipStream_t s) {
  k_pcg_residual<T><<<nb, kBlock, 0, s>>>(L, V, zero_x0 ? 1 : 0);
  k_pcg_start<T><<<nb, kBlock, 0, s>>>(L, V, sc, part);
}

template <typename T>
void launch_pcg_iter(const DLevel& L, const PcgVecs<T>& V, Scal* sc, double* part, int nb, int it,
                     double tol, bool check_only, hipStream_t s, hipEvent_t* ev) {
  if (ev) (void)hipEventRecord(ev[0], s);
  k_pcg_iter<T><<<nb, kBlock, 0, s>>>(L.n, V, sc, part, nb, it, tol, stamp(it, 1),
                                      check_only ? 1 : 0);
  if (ev) (void)hipEventRecord(ev[1], s);
}

void launch_make_ell(const DLevel& L, const double* val, const double* invd, int w,
                     int32_t* ell_col, double* ell_val, double* ell_sval, float* ell_sval32,
                     hipStream_t s) {
  k_make_ell<<<grid_for(L.n, kBlock), kBlock, 0, s>>>(L, val, invd, w, ell_col, ell_val, ell_sval,
                                                       ell_sval32);
}

template void launch_pcg_init<double>(const DLevel&, const PcgVecs<double>&, bool, Scal*, double*,
                                      int, hipStream_t);
template void launch_pcg_init<float>(const DLevel&, const PcgVecs<float>&, bool, Scal*, double*,
                                     int, hipStream_t);
template void launch_pcg_iter<double>(const DLevel&, const PcgVecs<double>&, Scal*, double*, int,
                                      int, double, bool, hipStream_t, hipEvent_t*);
template void launch_pcg_iter<float>(const DLevel&, const PcgVecs<float>&, Scal*, double*, int,
                                     int, double, bool, hipStream_t, hipEvent_t*);

void launch_restrict_galerkin(const int32_t* tri_f, int32_t n_fine_tris, const double2* xy_f,
                              int levels, const double* ut, int64_t stride, double* tripart,
                              hipStream_t s) {
  const int g = grid_for(n_fine_tris, kBlock);
  k_restrict_galerkin<<<g, kBlock, 0, s>>>(tri_f, n_fine_tris, xy_f, levels, ut, stride, tripart);
}

void launch_restrict_nodes(int32_t n_c, const int32_t* cn_ptr, const int32_t* cn_tri,
                           const double* tripart, const uint8_t* nat, double scale, double* b,
                           double* part, int nb, hipStream_t s) {
  k_restrict_nodes<<<nb, kBlock, 0, s>>>(n_c, cn_ptr, cn_tri, tripart, nat, scale, b, part);
}

void launch_restrict_inject(const DLevel& C, const uint8_t* nat, const double* ut,
                            int64_t stride, double scale, double* b, double* part, int nb,
                            hipStream_t s) {
  k_restrict_inject<<<nb, kBlock, 0, s>>>(C, nat, ut, stride, scale, b, part);
}

void launch_remove_mean(int32_t n, double* v, const double* part, int nb, const double* weights,
                        hipStream_t s) {
  k_remove_mean<<<nb, kBlock, 0, s>>>(n, v, part, nb, weights ? 1 : 0);
}

void launch_weighted_sums(int32_t n, const double* v, const double* w, double* part, int nb,
                          hipStream_t s) {
  k_weighted_sums<<<nb, kBlock, 0, s>>>(n, v, w, part);
}

void launch_prolong(int32_t n_f, const int32_t* pcode, const int32_t* tri_c, int levels,
                    const double* phic, double* phif, hipStream_t s) {
  k_prolong<<<grid_for(n_f, kBlock), kBlock, 0, s>>>(n_f, pcode, tri_c, levels, phic, phif);
}

void launch_correct_rhs(const DLevel& L, const int32_t* dir_index, const double* Mval,
                        double dt, double nu, int chi, int mass_mode, const double* phi_f,
                        const double* ut, const double* p_in, double* rhs, double* u_out,
                        double* p_out, const int32_t* lat_of, hipStream_t s) {
  k_correct_rhs<<<row_group_grid(L.n), kBlock, 0, s>>>(L, dir_index, Mval, dt, nu, chi, mass_mode,
                                                       phi_f, ut, p_in, rhs, u_out, p_out, lat_of);
}

void launch_final_update(int32_t n, const double* ut, const double* du, const double* p_in,
                         const double* phi_f, int nr, bool write_p, double* u_out,
                         double* p_out, const int32_t* lat_of, hipStream_t s) {
  k_final_update<<<grid_for(n, kBlock), kBlock, 0, s>>>(n, ut, du, p_in, phi_f, nr,
                                                        write_p ? 1 : 0, u_out, p_out, lat_of);
}

void launch_final_update2(int32_t n, const double* ut, const float* d1, const float* d2,
                          const double* p_in, const double* phi_f, int nr, bool write_p,
                          double* u_out, double* p_out, const int32_t* lat_of, hipStream_t s) {
  k_final_update2<<<grid_for(n, kBlock), kBlock, 0, s>>>(n, ut, d1, d2, p_in, phi_f, nr,
                                                         write_p ? 1 : 0, u_out, p_out, lat_of);
}

void launch_copy(const double* src, double* dst, int64_t n, hipStream_t s) {
  k_copy<<<grid_for(n, kBlock), kBlock, 0, s>>>(src, dst, n);
}
void launch_zero_masked(double* x, const uint8_t* nat, int32_t n, hipStream_t s) {
  k_zero_masked<<<grid_for(n, kBlock), kBlock, 0, s>>>(x, nat, n);
}
void launch_mirror(const Scal* src, Scal* host_dst, int n, hipStream_t s) {
  k_mirror<<<1, 64, 0, s>>>(src, host_dst, n);
}
void launch_axpy_f32(const float* d, double* x, int64_t n, hipStream_t s, const Scal* skip) {
  k_axpy_f32<<<grid_for(n, kBlock), kBlock, 0, s>>>(d, x, n, skip);
}
void launch_fill32(float* x, float v, int64_t n, hipStream_t s) {
  k_fill32<<<grid_for(n, kBlock), kBlock, 0, s>>>(x, v, n);
}
void launch_residual64(const DLevel& C, const double* Kval, const double* b, const double* x,
                       double* r, float* r32, double* part, int nb, hipStream_t s) {
  k_residual64<<<nb, kBlock, 0, s>>>(C, Kval, b, x, r, r32, part);
}
void launch_reduce_check(const double* part, int nb, double tol, Scal* sc, int outer,
                         hipStream_t s) {
  k_reduce_check<<<1, kBlock, 0, s>>>(part, nb, tol, sc, outer);
}

void launch_guard(const DLevel& C, const double* Kval, const double* b, const double* cand,
                  const double* prev, double* out, int32_t* chose, double* part, int nb,
                  hipStream_t s) {
  k_guard_residuals<<<nb, kBlock, 0, s>>>(C, Kval, b, cand, prev, part);
  k_guard_select<<<nb, kBlock, 0, s>>>(C.n, cand, prev, out, chose, part, nb);
}


void launch_fpcg_iter(int32_t n, const int32_t* ell_col, const double* ell_val, int ell_w,
                      const double* z, double* const p[2], double* q, double* x, double* r,
                      Scal* sc, double* part, int nb, int it, hipStream_t s, const Scal* skip) {
  k_fpcg_rz<<<nb, kBlock, 0, s>>>(n, r, z, part, skip);
  k_fpcg_dir<<<nb, kBlock, 0, s>>>(n, ell_col, ell_val, ell_w, z, p[(it - 1) & 1], p[it & 1], q,
                                   sc, part, nb, it, skip);
  k_fpcg_update<<<nb, kBlock, 0, s>>>(n, p[it & 1], q, x, r, sc, part, nb, it, skip);
}

void launch_fill(double* x, double v, int64_t n, hipStream_t s) {
  k_fill<<<grid_for(n, kBlock), kBlock, 0, s>>>(x, v, n);
}

}  // namespace cgp
