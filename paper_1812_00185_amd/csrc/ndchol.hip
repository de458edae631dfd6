// Triangular solves with the nested-dissection supernodal factor of K_c
// (layout in ndchol.hpp).  One work-group of one wave per item: a row range
// of G (forward) or a column range of G^T (backward), with the front vector
// of the supernode in LDS.  G is column-major, so for a fixed column the 64
// lanes read 64 consecutive rows.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ndchol.hpp"

namespace cgp {
namespace {

constexpr int kNdWave = 64;
static_assert(kNdItemRows == kNdWave, "one output row (column) per lane");

// forward: y_C and u of one item; f_C = r on C plus the children's updates
__global__ void __launch_bounds__(kNdWave)
k_nd_forward(NdDev d, const NdItem* __restrict__ items, const double* __restrict__ r) {
  extern __shared__ double fc[];
  const NdItem it = items[blockIdx.x];
  const NdSuper S = d.sn[it.sn];
  const int fs = S.w + S.m;
  for (int j = threadIdx.x; j < S.w; j += kNdWave) {
    double v = r[d.perm[S.c0 + j]];
    for (int q = d.gptr[S.gpos + j]; q < d.gptr[S.gpos + j + 1]; ++q) v += d.U[d.gidx[q]];
    fc[j] = v;
  }
  __syncthreads();
  const int o = it.lo + threadIdx.x;
  if (o >= it.hi) return;
  // rows of L11^-1 are zero right of the diagonal
  const int jmax = it.hi <= S.w ? it.hi : S.w;
  const double* __restrict__ g = d.G + S.goff + o;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int j = 0;
  for (; j + 4 <= jmax; j += 4) {
    a0 += g[(int64_t)j * fs] * fc[j];
    a1 += g[(int64_t)(j + 1) * fs] * fc[j + 1];
    a2 += g[(int64_t)(j + 2) * fs] * fc[j + 2];
    a3 += g[(int64_t)(j + 3) * fs] * fc[j + 3];
  }
  for (; j < jmax; ++j) a0 += g[(int64_t)j * fs] * fc[j];
  const double acc = (a0 + a1) + (a2 + a3);
  if (o < S.w) {
    d.Y[S.c0 + o] = acc;
  } else {
    double fr = 0.0;
    for (int q = d.gptr[S.gpos + o]; q < d.gptr[S.gpos + o + 1]; ++q) fr += d.U[d.gidx[q]];
    d.U[S.uoff + o - S.w] = fr - acc;
  }
}

// backward: x_C = G^T [y_C ; -x_R] for one item's columns
__global__ void __launch_bounds__(kNdWave)
k_nd_backward(NdDev d, const NdItem* __restrict__ items, double* __restrict__ z) {
  extern __shared__ double v[];
  const NdItem it = items[blockIdx.x];
  const NdSuper S = d.sn[it.sn];
  const int fs = S.w + S.m;
  // rows of the column range start at it.lo (L11^-T is upper triangular)
  for (int o = it.lo + threadIdx.x; o < fs; o += kNdWave)
    v[o] = o < S.w ? d.Y[S.c0 + o] : -d.X[d.rows[S.roff + o - S.w]];
  __syncthreads();
  const int i = it.lo + threadIdx.x;
  if (i >= it.hi) return;
  const double* __restrict__ g = d.GT + S.goff + i;
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  int o = it.lo;
  for (; o + 4 <= fs; o += 4) {
    a0 += g[(int64_t)o * S.w] * v[o];
    a1 += g[(int64_t)(o + 1) * S.w] * v[o + 1];
    a2 += g[(int64_t)(o + 2) * S.w] * v[o + 2];
    a3 += g[(int64_t)(o + 3) * S.w] * v[o + 3];
  }
  for (; o < fs; ++o) a0 += g[(int64_t)o * S.w] * v[o];
  const double acc = (a0 + a1) + (a2 + a3);
  d.X[S.c0 + i] = acc;
  z[d.perm[S.c0 + i]] = acc;
}

}  // namespace

void launch_nd_solve(const NdDev& d, const NdFactor& f, const double* r, double* z,
                     hipStream_t s) {
  for (int L = 0; L < f.height; ++L) {
    const int a = f.fwd_lvl[L], b = f.fwd_lvl[L + 1];
    int lds = 1;
    for (int k = a; k < b; ++k) lds = std::max(lds, f.sn[f.fwd[k].sn].w);
    k_nd_forward<<<b - a, kNdWave, sizeof(double) * lds, s>>>(d, d.fwd + a, r);
  }
  for (int q = 0; q < f.height; ++q) {
    const int a = f.bwd_lvl[q], b = f.bwd_lvl[q + 1];
    int lds = 1;
    for (int k = a; k < b; ++k) lds = std::max(lds, f.sn[f.bwd[k].sn].w + f.sn[f.bwd[k].sn].m);
    k_nd_backward<<<b - a, kNdWave, sizeof(double) * lds, s>>>(d, d.bwd + a, z);
  }
}

}  // namespace cgp
