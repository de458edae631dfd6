// Nested-dissection supernodal Cholesky factor of the coarse Poisson matrix,
// used as the preconditioner of the coarse PCG (host set-up; the solves run in
// ndchol.hip).
//
// K_c never changes during a run, so it is factored once.  The unknowns (the
// coarse nodes minus the phi = 0 nodes, and minus one pinned node when no
// boundary is natural and K_c is singular) are ordered by geometric nested
// dissection of the node coordinates: a node set larger than the leaf size is
// split at the median of its longer bounding-box side, the nodes of the first
// half that touch the second half form the separator, and the two remaining
// parts are ordered recursively before it.  Every leaf and every separator is
// one supernode (a contiguous range of columns), in post-order.
//
// Supernode s has columns C (width w) and below-diagonal row set R (m rows,
// ancestors' columns only).  The multifrontal factorisation gives the dense
// blocks L11 (w x w) and L21 (m x w) of L, L L^T = K (permuted).  Stored per
// supernode is G = [L11^-1 ; L21 L11^-1] ((w + m) x w, column-major) and its
// transpose, so that both triangular solves become dense products:
//   forward   [y_C ; t] = G f_C,  u = f_R - t       (f: front vector)
//   backward  x_C = G^T [y_C ; -x_R]
// where the front vector of s is r on C plus the update vectors u of its
// children, scattered to their positions in C and R.  Supernodes of one tree
// level are independent, so each direction is one launch per level.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace cgp {

struct NdSuper {
  int32_t c0, w, m;  // first column (ND position), width, below-diagonal rows
  int32_t level;     // 0 for leaves, 1 + max over children otherwise
  int64_t goff;      // offset of G (and of G^T) in the factor arrays
  int32_t roff;      // offset of R in `rows`
  int32_t uoff;      // offset of the update vector u in the update buffer
  int32_t gpos;      // offset of the first front position in `gptr`
};

// One work-group's share of a level: forward items are row ranges [lo, hi)
// of G, backward items column ranges of G^T.
struct NdItem {
  int32_t sn, lo, hi;
};

struct NdFactor {
  int32_t n = 0;                  // matrix size (coarse nodes)
  int32_t nfac = 0;               // factored unknowns
  std::vector<int32_t> perm;      // [nfac] ND position -> node
  std::vector<int32_t> pos;       // [n] node -> ND position or -1
  std::vector<NdSuper> sn;        // post-order
  std::vector<std::vector<int32_t>> children;
  std::vector<int32_t> rows;      // R of every supernode (ND positions, ascending)
  // for every front position of every supernode, the update-vector entries
  // of its children that add into it (CSR over positions)
  std::vector<int32_t> gptr, gidx;
  int64_t g_entries = 0;          // sum over supernodes of (w + m) w
  int32_t n_upd = 0;              // total update-vector length
  int32_t height = 0;             // tree levels
  int32_t max_w = 0, max_front = 0;
  std::vector<NdItem> fwd, bwd;   // grouped by level (forward: leaves first)
  std::vector<int32_t> fwd_lvl, bwd_lvl;  // [height + 1] item offsets per level
  std::vector<double> G, GT;      // numeric factor
};

constexpr int kNdLeaf = 32;       // leaf size of the dissection
constexpr int kNdItemRows = 64;   // rows (forward) / columns (backward) per item
constexpr int kNdMaxFront = 8192; // LDS bound: front vector of doubles <= 64 KiB

// Ordering and structure.  skip[i] != 0 removes node i (its solution entry is
// 0).  Returns "" on success.
std::string nd_symbolic(int32_t n, const std::vector<int32_t>& rowptr,
                        const std::vector<int32_t>& col, const double* xy,
                        const std::vector<uint8_t>& skip, NdFactor& f);

// Numeric factorisation of the symmetric matrix with the given CSR values
// (only the rows and columns that are not skipped are read; the lower
// triangle in ND order is used).  Returns "" on success, else the reason (a
// non-positive pivot: the matrix is not positive definite there).
std::string nd_numeric(const std::vector<int32_t>& rowptr, const std::vector<int32_t>& col,
                       const double* val, NdFactor& f);

// z = K^-1 r on the factored unknowns (0 elsewhere), by the same level
// algorithm as the device kernels.
void nd_solve_host(const NdFactor& f, const double* r, double* z);

}  // namespace cgp

#include <hip/hip_runtime.h>

namespace cgp {

// Device copy of a factor (arrays in the caller's workspace), with the
// factor entries, front vectors and results of type T: double for the FP64
// coarse solve, float for the FP32 solve inside the mixed-precision
// refinement (FP32 storage and FP32 accumulation).
template <typename T>
struct NdDevT {
  int32_t nfac;
  const int32_t* perm;
  const NdSuper* sn;
  const int32_t* rows;
  const int32_t* gptr;
  const int32_t* gidx;
  const NdItem* fwd;
  const NdItem* bwd;
  const T* G;
  const T* GT;
  T* Y;  // [nfac] forward result
  T* X;  // [nfac] backward result (ND order)
  T* U;  // [n_upd] update vectors
};
using NdDev = NdDevT<double>;
using NdDev32 = NdDevT<float>;

struct Scal;

// z = K^-1 r on the factored unknowns: one forward launch per tree level
// (leaves first), then one backward launch per level (root first).  Entries
// of z at skipped nodes are not written.  With skip_if_done != nullptr every
// launch returns at once when that record's done_stamp is set.
template <typename T>
void launch_nd_solve(const NdDevT<T>& d, const NdFactor& f, const T* r, T* z, hipStream_t s,
                     const Scal* skip_if_done = nullptr);

}  // namespace cgp
