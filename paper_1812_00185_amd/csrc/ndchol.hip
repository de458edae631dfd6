// Triangular solves with the nested-dissection supernodal factor of K_c
// (layout in ndchol.hpp).  One work-group per item: a row range of G
// (forward) or a column range of G^T (backward), with the front vector of the
// supernode in LDS.  G is column-major, so for a fixed column the 64 lanes of
// a wave read 64 consecutive rows; the W waves of the group split the
// reduction range.  A level's launch takes W (4, 8 or 16) from its longest
// reduction, so that a wave walks at most 16 terms (8 loads in flight each)
// for reductions of up to 256 terms and len / 16 beyond, and the wide
// separators near the root are not a long chain of dependent loads.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "device.hpp"
#include "ndchol.hpp"

namespace cgp {
namespace {

constexpr int kNdWave = 64;
static_assert(kNdItemRows == kNdWave, "one output row (column) per lane");

// sum over [a, b) of g[k * ld] * x[k], 8 loads in flight (accumulated in T)
template <typename T>
__device__ __forceinline__ T dot_strided(const T* __restrict__ g, int64_t ld, const T* x, int a,
                                         int b) {
  T acc[8] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
  int k = a;
  for (; k + 8 <= b; k += 8) {
#pragma unroll
    for (int u = 0; u < 8; ++u) acc[u] += g[(int64_t)(k + u) * ld] * x[k + u];
  }
  for (; k < b; ++k) acc[0] += g[(int64_t)k * ld] * x[k];
  return ((acc[0] + acc[1]) + (acc[2] + acc[3])) + ((acc[4] + acc[5]) + (acc[6] + acc[7]));
}

// the W partial sums of each lane, added in wave order by wave 0
template <typename T, int W>
__device__ __forceinline__ T combine(T part, T (&sh)[W][kNdWave]) {
  const int lane = threadIdx.x % kNdWave, wv = threadIdx.x / kNdWave;
  sh[wv][lane] = part;
  __syncthreads();
  T t = T(0);
  if (wv == 0) {
#pragma unroll
    for (int q = 0; q < W; ++q) t += sh[q][lane];
  }
  return t;
}

__device__ __forceinline__ bool nd_skip(const Scal* flag) {
  return flag != nullptr && flag->done_stamp != 0;
}

// forward: y_C and u of one item; f_C = r on C plus the children's updates
template <typename T, int W>
__global__ void __launch_bounds__(W * kNdWave)
k_nd_forward(NdDevT<T> d, const NdItem* __restrict__ items, const T* __restrict__ r,
             const Scal* flag) {
  extern __shared__ __align__(16) unsigned char fc_raw[];
  T* fc = reinterpret_cast<T*>(fc_raw);
  __shared__ T part[W][kNdWave];
  if (nd_skip(flag)) return;
  const NdItem it = items[blockIdx.x];
  const NdSuper S = d.sn[it.sn];
  const int fs = S.w + S.m;
  for (int j = threadIdx.x; j < S.w; j += W * kNdWave) {
    T v = r[d.perm[S.c0 + j]];
    for (int q = d.gptr[S.gpos + j]; q < d.gptr[S.gpos + j + 1]; ++q) v += d.U[d.gidx[q]];
    fc[j] = v;
  }
  __syncthreads();
  const int lane = threadIdx.x % kNdWave, wv = threadIdx.x / kNdWave;
  const int o = it.lo + lane;
  const int oc = o < it.hi ? o : it.lo;  // idle lanes read a valid row
  // rows of L11^-1 are zero right of the diagonal
  const int jmax = it.hi <= S.w ? it.hi : S.w;
  const int chunk = (jmax + W - 1) / W;
  const int a = min(jmax, wv * chunk), b = min(jmax, a + chunk);
  const T acc = combine<T, W>(dot_strided<T>(d.G + S.goff + oc, fs, fc, a, b), part);
  if (wv != 0 || o >= it.hi) return;
  if (o < S.w) {
    d.Y[S.c0 + o] = acc;
  } else {
    T fr = T(0);
    for (int q = d.gptr[S.gpos + o]; q < d.gptr[S.gpos + o + 1]; ++q) fr += d.U[d.gidx[q]];
    d.U[S.uoff + o - S.w] = fr - acc;
  }
}

// backward: x_C = G^T [y_C ; -x_R] for one item's columns
template <typename T, int W>
__global__ void __launch_bounds__(W * kNdWave)
k_nd_backward(NdDevT<T> d, const NdItem* __restrict__ items, T* __restrict__ z,
              const Scal* flag) {
  extern __shared__ __align__(16) unsigned char v_raw[];
  T* v = reinterpret_cast<T*>(v_raw);
  __shared__ T part[W][kNdWave];
  if (nd_skip(flag)) return;
  const NdItem it = items[blockIdx.x];
  const NdSuper S = d.sn[it.sn];
  const int fs = S.w + S.m;
  // rows of the column range start at it.lo (L11^-T is upper triangular)
  for (int o = it.lo + threadIdx.x; o < fs; o += W * kNdWave)
    v[o] = o < S.w ? d.Y[S.c0 + o] : -d.X[d.rows[S.roff + o - S.w]];
  __syncthreads();
  const int lane = threadIdx.x % kNdWave, wv = threadIdx.x / kNdWave;
  const int i = it.lo + lane;
  const int ic = i < it.hi ? i : it.lo;
  const int len = fs - it.lo;
  const int chunk = (len + W - 1) / W;
  const int a = it.lo + min(len, wv * chunk), b = it.lo + min(len, (wv + 1) * chunk);
  const T acc = combine<T, W>(dot_strided<T>(d.GT + S.goff + ic, S.w, v, a, b), part);
  if (wv != 0 || i >= it.hi) return;
  d.X[S.c0 + i] = acc;
  z[d.perm[S.c0 + i]] = acc;
}

}  // namespace

// waves per item for a level whose longest reduction has len terms
inline int nd_waves(int len) { return len <= 64 ? 4 : (len <= 128 ? 8 : 16); }

template <typename T, int W>
void nd_forward(const NdDevT<T>& d, int a, int b, int lds, const T* r, hipStream_t s,
                const Scal* skip_if_done) {
  k_nd_forward<T, W><<<b - a, W * kNdWave, sizeof(T) * lds, s>>>(d, d.fwd + a, r, skip_if_done);
}

template <typename T, int W>
void nd_backward(const NdDevT<T>& d, int a, int b, int lds, T* z, hipStream_t s,
                 const Scal* skip_if_done) {
  k_nd_backward<T, W><<<b - a, W * kNdWave, sizeof(T) * lds, s>>>(d, d.bwd + a, z, skip_if_done);
}

template <typename T>
void launch_nd_solve(const NdDevT<T>& d, const NdFactor& f, const T* r, T* z, hipStream_t s,
                     const Scal* skip_if_done) {
  for (int L = 0; L < f.height; ++L) {
    const int a = f.fwd_lvl[L], b = f.fwd_lvl[L + 1];
    int lds = 1, len = 0;
    for (int k = a; k < b; ++k) {
      const NdItem& it = f.fwd[k];
      const NdSuper& S = f.sn[it.sn];
      lds = std::max(lds, S.w);
      len = std::max(len, std::min(it.hi, S.w));
    }
    const int W = nd_waves(len);
    if (W == 4)
      nd_forward<T, 4>(d, a, b, lds, r, s, skip_if_done);
    else if (W == 8)
      nd_forward<T, 8>(d, a, b, lds, r, s, skip_if_done);
    else
      nd_forward<T, 16>(d, a, b, lds, r, s, skip_if_done);
  }
  for (int q = 0; q < f.height; ++q) {
    const int a = f.bwd_lvl[q], b = f.bwd_lvl[q + 1];
    int lds = 1, len = 0;
    for (int k = a; k < b; ++k) {
      const NdItem& it = f.bwd[k];
      const NdSuper& S = f.sn[it.sn];
      lds = std::max(lds, S.w + S.m);
      len = std::max(len, S.w + S.m - it.lo);
    }
    const int W = nd_waves(len);
    if (W == 4)
      nd_backward<T, 4>(d, a, b, lds, z, s, skip_if_done);
    else if (W == 8)
      nd_backward<T, 8>(d, a, b, lds, z, s, skip_if_done);
    else
      nd_backward<T, 16>(d, a, b, lds, z, s, skip_if_done);
  }
}

template void launch_nd_solve<double>(const NdDevT<double>&, const NdFactor&, const double*,
                                      double*, hipStream_t, const Scal*);
template void launch_nd_solve<float>(const NdDevT<float>&, const NdFactor&, const float*,
                                     float*, hipStream_t, const Scal*);

}  // namespace cgp
