// Mass-matrix solves of the velocity correction and the rotational pressure
// update (Eqs. 25-26) on the lattice layout of lattice.hpp.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "cheb2.hpp"
#include "corrlat.hpp"
#include "device.hpp"
#include "lattice.hpp"

namespace cgp {
namespace {

// ------------------------------------------------------------------ Chebyshev
// Mass-matrix solves M x = b on NR right-hand sides at once (the first two
// with the Dirichlet rows removed, a third -- the rotational pressure update --
// on all rows).  The Jacobi-scaled P1 mass matrix has its spectrum in
// [1/2, 2], so Chebyshev acceleration on that interval needs no inner
// products: x_{k+1} = x_k + a_k (x_k - x_{k-1}) + c_k D^-1 (b - M x_k), one
// fused kernel per iteration with the iterates in three rotating buffers.
// Right-hand sides and iterates are interleaved per node ([n][NR]) so that a
// gathered neighbour costs one contiguous access.
//
// One Chebyshev step of the mass solves on the lattice layout (one thread per
// lattice node): x_new = x_k + ca (x_k - x_{k-1}) + cb D^-1 (b - M x_k), the
// velocity components held at 0 on Dirichlet nodes.  M x_k and D come from
// the lattice stencils (no matrix read away from the coarse vertices).  The
// first step (x_0 = 0) needs only D and also clears x_k, which the next step
// reads back as x_{k-1}.
//
// Memory access: a block's 256 nodes own a contiguous range of 256 NR
// doubles in every vector.  The block moves its ranges of b, x_{k-1}, x_k
// (read) and x_new (written) between HBM and LDS as contiguous 16-byte
// pieces, so these streams cost whole cache lines per instruction instead of
// NR strided 8-byte accesses per node (on MI355X the strided form measured
// 169 us per launch against 127 us staged, 2049^2 k = 3, NR = 3); neighbours
// inside the block's range are read from LDS, the others gathered from x_k.
// b and the iterates must be 16-byte aligned (the workspace pieces are
// 256-byte aligned).  The launch covers the nodes [lbase, n), lbase a multiple
// of 4 (so that every block range starts 16-byte aligned), with
// (n - lbase) / kBlock blocks rounded up.  Values are stored as T (double, or
// float for the inner solves of the mixed-precision form) and combined in
// FP64.
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ inline void ld16(const T* src, T* dst) {
  *reinterpret_cast<u32x4*>(dst) = *reinterpret_cast<const u32x4*>(src);
}
template <typename T>
__device__ inline void ldnt16(const T* src, T* dst) {
  *reinterpret_cast<u32x4*>(dst) = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(src));
}
template <typename T>
__device__ inline void stnt16(const T* src, T* dst) {
  __builtin_nontemporal_store(*reinterpret_cast<const u32x4*>(src), reinterpret_cast<u32x4*>(dst));
}

template <typename T, int NR, int M>
__global__ void __launch_bounds__(kBlock)
k_cheb_lattice(LatDev L, int32_t n, int32_t lbase, const T* __restrict__ b, T* __restrict__ xk,
               const T* __restrict__ xkm, T* __restrict__ xnew, double ca, double cb, int first) {
  constexpr int kPer = 16 / (int)sizeof(T);  // values per 16-byte piece
  constexpr int kVals = kBlock * NR;         // values per block
  constexpr int kPieces = kVals / kPer;
  static_assert(kVals % kPer == 0, "block range in whole pieces");
  __shared__ u32x4 sb[kPieces], sm[kPieces], sx[kPieces];
  T* sbd = reinterpret_cast<T*>(sb);
  T* smd = reinterpret_cast<T*>(sm);
  T* sxd = reinterpret_cast<T*>(sx);
  // blocks in reverse order: the coarse-vertex rows (at the end of the
  // layout; short rows of dependent gathers) start first instead of trailing
  const int32_t l0 = lbase + (int32_t)(gridDim.x - 1 - blockIdx.x) * kBlock;
  const int32_t l = l0 + threadIdx.x;
  const int64_t v0 = (int64_t)l0 * NR;   // first value of the block
  const int64_t vend = (int64_t)n * NR;  // values in the vector
#pragma unroll
  for (int q = threadIdx.x; q < kPieces; q += kBlock) {
    const int64_t v = v0 + (int64_t)q * kPer;
    if (v + kPer <= vend) {
      // b and x_{k-1} are read once per launch: non-temporal, so that the L2
      // keeps x_k, which neighbouring blocks gather
      ldnt16(b + v, sbd + q * kPer);
      if (!first) {
        ldnt16(xkm + v, smd + q * kPer);
        ld16(xk + v, sxd + q * kPer);
      }
    } else {
#pragma unroll
      for (int j = 0; j < kPer; ++j)
        if (v + j < vend) {
          sbd[q * kPer + j] = b[v + j];
          if (!first) {
            smd[q * kPer + j] = xkm[v + j];
            sxd[q * kPer + j] = xk[v + j];
          }
        }
    }
  }
  __syncthreads();
  double out[NR];
  if (l < n) {
    const bool masked = L.ldir[l] != 0;
    const int t = threadIdx.x * NR;
    if (first) {
      const double di = 1.0 / lat_diag(L, l);
#pragma unroll
      for (int d = 0; d < NR; ++d) out[d] = (d < 2 && masked) ? 0.0 : cb * di * (double)sbd[t + d];
    } else {
      double y[NR], diag;
      // neighbours inside the block's range come from LDS
      auto xv = [&](int32_t i, int d) {
        const uint32_t r = (uint32_t)(i - l0);
        return r < (uint32_t)kBlock ? (double)sxd[r * NR + d] : (double)xk[(int64_t)i * NR + d];
      };
      lat_apply<NR, M>(L, l, xv, y, diag);
      const double di = 1.0 / diag;
#pragma unroll
      for (int d = 0; d < NR; ++d) {
        const double xv = sxd[t + d];
        out[d] = (d < 2 && masked) ? 0.0 : xv + ca * (xv - (double)smd[t + d]) + cb * di * ((double)sbd[t + d] - y[d]);
      }
    }
  }
  __syncthreads();  // every read of sm is done: it now stages x_new
  if (l < n) {
#pragma unroll
    for (int d = 0; d < NR; ++d) smd[threadIdx.x * NR + d] = (T)out[d];
  }
  __syncthreads();
#pragma unroll
  for (int q = threadIdx.x; q < kPieces; q += kBlock) {
    const int64_t v = v0 + (int64_t)q * kPer;
    if (v + kPer <= vend) {
      stnt16(smd + q * kPer, xnew + v);
      if (first) *reinterpret_cast<u32x4*>(xk + v) = u32x4{0u, 0u, 0u, 0u};
    } else {
#pragma unroll
      for (int j = 0; j < kPer; ++j)
        if (v + j < vend) {
          xnew[v + j] = smd[q * kPer + j];
          if (first) xk[v + j] = (T)0;
        }
    }
  }
}

// r = b - M x over every lattice node, b in FP64 and x stored as float, r
// (FP64 arithmetic) stored as float; velocity components 0 at Dirichlet
// nodes (the refinement residual of the mixed-precision mass solves).  One
// thread per node, plain loads: staging x's block range through LDS (with
// non-temporal loads of b) measured slower, 72 -> 83 us at 2049^2.
template <int NR, int M>
__global__ void __launch_bounds__(kBlock)
k_mass_resid(LatDev L, int32_t n, const double* __restrict__ b, const float* __restrict__ x,
             float* __restrict__ r) {
  const int32_t l = blockIdx.x * kBlock + threadIdx.x;
  if (l >= n) return;
  double y[NR], diag;
  lat_apply<NR, M>(L, l, [&](int32_t i, int d) { return (double)x[(int64_t)i * NR + d]; }, y,
                   diag);
  const bool masked = L.ldir[l] != 0;
#pragma unroll
  for (int d = 0; d < NR; ++d)
    r[(int64_t)l * NR + d] = (d < 2 && masked) ? 0.0f : (float)(b[(int64_t)l * NR + d] - y[d]);
}

// neighbour table of the interior stencil (cheb2.hpp), in constant memory
__constant__ Ch2NbTable kCh2NbDev = ch2_make_nb_table();

// Two Chebyshev steps on the interior nodes of kCh2Tris coarse triangles per
// block (lattice size 8; the phases and their data flow are in cheb2.hpp).
// 36 KB of LDS per block for T = double, NR = 3.
template <typename T, int NR>
__global__ void __launch_bounds__(kCh2Threads) k_cheb_pair(LatDev L, Cheb2Args<T> A) {
  __shared__ __align__(16) Cheb2Shared<T, NR> S;
  const int blk = blockIdx.x, tid = threadIdx.x;
  auto ld = [](const T* src, T* dst) { ld16(src, dst); };
  auto ldnt = [](const T* src, T* dst) { ldnt16(src, dst); };
  auto stnt = [](const T* src, T* dst) { stnt16(src, dst); };
  ch2_stage<T, NR>(L, A, blk, tid, S, ld, ldnt);
  __syncthreads();
  ch2_step1<T, NR>(L, A, blk, tid, kCh2NbDev.w, S);
  __syncthreads();
  ch2_step2<T, NR>(L, A, blk, tid, kCh2NbDev.w, S);
  __syncthreads();
  ch2_write<T, NR>(L, A, blk, tid, S, stnt);
}

// Right-hand sides of the consistent-mass solves on the lattice layout (one
// thread per lattice node; the stencils are in corrlat.hpp): rhs [n][NR],
// NR = 2 + chi, written through LDS as 16-byte pieces of the block's range.
// With rhs32 (not null) also a float copy, the right-hand side of the first
// inner solve of the mixed-precision form.
template <int NR, int M, bool kPc>
__global__ void __launch_bounds__(kBlock) k_correct_rhs_lat(LatDev L, CorrLatArgs A,
                                                            double* __restrict__ rhs,
                                                            float* __restrict__ rhs32) {
  constexpr int kPieces = kBlock * NR / 2;
  __shared__ double2 so[kPieces];
  double* sod = reinterpret_cast<double*>(so);
  const int32_t n = A.n;
  const int32_t l0 = blockIdx.x * kBlock;
  const int32_t l = l0 + threadIdx.x;
  if (l < n) {
    double out[3];
    corr_node<M, kPc>(L, A, l, out);
#pragma unroll
    for (int d = 0; d < NR; ++d) sod[threadIdx.x * NR + d] = out[d];
  }
  __syncthreads();
  const int64_t v0 = (int64_t)l0 * NR, vend = (int64_t)n * NR;
  double2* o2 = reinterpret_cast<double2*>(rhs + v0);
  for (int q = threadIdx.x; q < kPieces; q += kBlock) {
    if (v0 + 2 * q + 1 < vend)
      o2[q] = so[q];
    else if (v0 + 2 * q < vend)
      rhs[v0 + 2 * q] = sod[2 * q];
  }
  if (rhs32) {
    float2* f2 = reinterpret_cast<float2*>(rhs32 + v0);
    for (int q = threadIdx.x; q < kPieces; q += kBlock) {
      if (v0 + 2 * q + 1 < vend)
        f2[q] = make_float2((float)sod[2 * q], (float)sod[2 * q + 1]);
      else if (v0 + 2 * q < vend)
        rhs32[v0 + 2 * q] = (float)sod[2 * q];
    }
  }
}

__global__ void __launch_bounds__(kBlock)
k_corr_gather(int32_t n, const int32_t* __restrict__ node_of, const double* __restrict__ phi,
              const double* __restrict__ ut, double* __restrict__ v4) {
  const int32_t l = blockIdx.x * kBlock + threadIdx.x;
  if (l < n) corr_gather(n, node_of, phi, ut, l, v4);
}

}  // namespace

bool launch_correct_rhs_lattice(const LatDev& L, const int32_t* node_of, const double* phi,
                                const double* ut, const CorrLatArgs& A, double* rhs,
                                float* rhs32, hipStream_t s) {
  if (((uintptr_t)rhs & 15) != 0 || ((uintptr_t)A.v4 & 15) != 0 || ((uintptr_t)rhs32 & 7) != 0)
    return false;
  const int g = (A.n + kBlock - 1) / kBlock;
  if (!lat_dispatch(L.m, [](auto) {})) return false;
  // with phi_c the copy holds U~ only
  k_corr_gather<<<g, kBlock, 0, s>>>(A.n, node_of, A.phi_c ? nullptr : phi, ut,
                                     const_cast<double*>(A.v4));
  return lat_dispatch(L.m, [&](auto lat) {
    constexpr int M = decltype(lat)::kM;
    if (A.phi_c) {
      if (A.chi)
        k_correct_rhs_lat<3, M, true><<<g, kBlock, 0, s>>>(L, A, rhs, rhs32);
      else
        k_correct_rhs_lat<2, M, true><<<g, kBlock, 0, s>>>(L, A, rhs, rhs32);
    } else if (A.chi) {
      k_correct_rhs_lat<3, M, false><<<g, kBlock, 0, s>>>(L, A, rhs, rhs32);
    } else {
      k_correct_rhs_lat<2, M, false><<<g, kBlock, 0, s>>>(L, A, rhs, rhs32);
    }
  });
}

int cheb_iterations(double tol) {
  // error reduction 2 ((sqrt(k)-1)/(sqrt(k)+1))^m with k = 4 (interval [1/2, 2]),
  // times sqrt(k) from the energy norm to the scaled residual
  const double rate = 1.0 / 3.0;
  int m = (int)std::ceil(std::log(4.0 / tol) / std::log(1.0 / rate));
  return m < 1 ? 1 : m;
}

namespace {

// The solve of launch_cheb for iterates stored as T.
template <typename T>
T* cheb_solve(const LatDev& L, int32_t n, const T* b, int nr, T* const x[3], int iters,
              hipStream_t s, hipEvent_t* (*timer)(void*, int), void* tctx) {
  // the kernels move their block ranges as 16-byte pieces
  const uintptr_t align = (uintptr_t)b | (uintptr_t)x[0] | (uintptr_t)x[1] | (uintptr_t)x[2];
  if ((align & 15) != 0 || !lat_dispatch(L.m, [](auto) {})) return nullptr;
  const double lo = 0.5, hi = 2.0;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  // step k: (ca_k, cb_k) of the three-term recurrence
  double rho = 1.0 / sigma;
  auto coef = [&](int k, double& ca, double& cb) {
    ca = 0.0;
    cb = 1.0 / theta;
    if (k > 0) {
      const double rn = 1.0 / (2.0 * sigma - rho);
      ca = rn * rho;
      cb = 2.0 * rn / delta;
      rho = rn;
    }
  };
  // single step k over the nodes [lbase, n); x_k in x[k % 3], x_{k-1} in
  // x[(k + 2) % 3], x_{k+1} into x[(k + 1) % 3]
  auto single = [&](int k, int32_t lbase, double ca, double cb) {
    const int g = (n - lbase + kBlock - 1) / kBlock;
    if (g <= 0) return;
    T* xk = x[k % 3];
    const T* xkm = x[(k + 2) % 3];
    T* xn = x[(k + 1) % 3];
    hipEvent_t* ev = (timer && k > 0) ? timer(tctx, kChebTimedSingle) : nullptr;
    if (ev) (void)hipEventRecord(ev[0], s);
    lat_dispatch(L.m, [&](auto lat) {
      constexpr int M = decltype(lat)::kM;
      if (nr == 3)
        k_cheb_lattice<T, 3, M><<<g, kBlock, 0, s>>>(L, n, lbase, b, xk, xkm, xn, ca, cb, k == 0);
      else
        k_cheb_lattice<T, 2, M><<<g, kBlock, 0, s>>>(L, n, lbase, b, xk, xkm, xn, ca, cb, k == 0);
    });
    if (ev) (void)hipEventRecord(ev[1], s);
  };
  // steps in pairs on lattice size 8: edge and vertex nodes (from the node
  // at or below EB with an index divisible by 4, so that block ranges start
  // 16-byte aligned), the interior two steps at once, edge and vertex nodes
  // again
  const bool pairs = L.m == kCh2M && L.nT > 0 && L.EB == L.nT * kCh2NI;
  const int32_t lb = L.EB & ~3;
  const int gp = (L.nT + kCh2Tris - 1) / kCh2Tris;
  double ca, cb;
  coef(0, ca, cb);
  single(0, 0, ca, cb);
  for (int k = 1; k < iters;) {
    coef(k, ca, cb);
    if (!pairs || k + 1 >= iters) {
      single(k, 0, ca, cb);
      k += 1;
      continue;
    }
    double ca2, cb2;
    coef(k + 1, ca2, cb2);
    single(k, lb, ca, cb);
    const Cheb2Args<T> A{n, b, x[(k + 2) % 3], x[k % 3], x[(k + 1) % 3], x[(k + 2) % 3],
                         ca, cb, ca2, cb2};
    hipEvent_t* ev = timer ? timer(tctx, kChebTimedPair) : nullptr;
    if (ev) (void)hipEventRecord(ev[0], s);
    if (nr == 3)
      k_cheb_pair<T, 3><<<gp, kCh2Threads, 0, s>>>(L, A);
    else
      k_cheb_pair<T, 2><<<gp, kCh2Threads, 0, s>>>(L, A);
    if (ev) (void)hipEventRecord(ev[1], s);
    single(k + 1, lb, ca2, cb2);
    k += 2;
  }
  return x[iters % 3];
}

}  // namespace

double* launch_cheb(const LatDev& L, int32_t n, const double* b, int nr,
                    double* const x[3], int iters, hipStream_t s,
                    hipEvent_t* (*timer)(void*, int), void* tctx) {
  return cheb_solve<double>(L, n, b, nr, x, iters, s, timer, tctx);
}

bool launch_cheb_mixed(const LatDev& L, int32_t n, const double* b, int nr, float* const y[5],
                       int iters, hipStream_t s, hipEvent_t* (*timer)(void*, int), void* tctx,
                       const float** d1, const float** d2) {
  if (!lat_dispatch(L.m, [](auto) {})) return false;
  // first inner solve: M d1 = b (float copy in y[3])
  float* const x1[3] = {y[0], y[1], y[2]};
  float* r1 = cheb_solve<float>(L, n, y[3], nr, x1, iters, s, timer, tctx);
  if (!r1) return false;
  // refinement residual r = b - M d1 over b's float copy
  const int g = (n + kBlock - 1) / kBlock;
  lat_dispatch(L.m, [&](auto lat) {
    constexpr int M = decltype(lat)::kM;
    if (nr == 3)
      k_mass_resid<3, M><<<g, kBlock, 0, s>>>(L, n, b, r1, y[3]);
    else
      k_mass_resid<2, M><<<g, kBlock, 0, s>>>(L, n, b, r1, y[3]);
  });
  // second inner solve M d2 = r, in the buffers d1 does not occupy
  float* x2[3];
  int j = 0;
  for (int k = 0; k < 3; ++k)
    if (y[k] != r1) x2[j++] = y[k];
  x2[2] = y[4];
  float* r2 = cheb_solve<float>(L, n, y[3], nr, x2, iters, s, timer, tctx);
  if (!r2) return false;
  *d1 = r1;
  *d2 = r2;
  return true;
}

}  // namespace cgp
