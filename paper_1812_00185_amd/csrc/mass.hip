// Mass-matrix solves of the velocity correction and the rotational pressure
// update (Eqs. 25-26) on the lattice layout of lattice.hpp.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

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
// 256-byte aligned).
typedef double nt_d2 __attribute__((ext_vector_type(2)));

template <int NR, int M>
__global__ void __launch_bounds__(kBlock)
k_cheb_lattice(LatDev L, int32_t n, const double* __restrict__ b, double* __restrict__ xk,
               const double* __restrict__ xkm, double* __restrict__ xnew, double ca, double cb,
               int first) {
  constexpr int kVals = kBlock * NR;  // doubles per block
  constexpr int kPieces = kVals / 2;  // 16-byte pieces per block
  __shared__ double2 sb[kPieces], sm[kPieces], sx[kPieces];
  const int32_t l0 = blockIdx.x * kBlock;
  const int32_t l = l0 + threadIdx.x;
  const int64_t v0 = (int64_t)l0 * NR;  // first double of the block
  const int64_t vend = (int64_t)n * NR;  // doubles in the vector
  const double2* b2 = reinterpret_cast<const double2*>(b + v0);
  const double2* m2 = reinterpret_cast<const double2*>(xkm + v0);
  const double2* x2 = reinterpret_cast<const double2*>(xk + v0);
#pragma unroll
  for (int q = threadIdx.x; q < kPieces; q += kBlock) {
    if (v0 + 2 * q + 1 < vend) {
      // b and x_{k-1} are read once per launch: non-temporal, so that the L2
      // keeps x_k, which neighbouring blocks gather
      const nt_d2 bv = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(b2) + q);
      sb[q] = make_double2(bv.x, bv.y);
      if (!first) {
        const nt_d2 mv = __builtin_nontemporal_load(reinterpret_cast<const nt_d2*>(m2) + q);
        sm[q] = make_double2(mv.x, mv.y);
        sx[q] = x2[q];
      }
    } else if (v0 + 2 * q < vend) {
      sb[q] = make_double2(b[v0 + 2 * q], 0.0);
      if (!first) {
        sm[q] = make_double2(xkm[v0 + 2 * q], 0.0);
        sx[q] = make_double2(xk[v0 + 2 * q], 0.0);
      }
    }
  }
  __syncthreads();
  const double* sbd = reinterpret_cast<const double*>(sb);
  const double* smd = reinterpret_cast<const double*>(sm);
  const double* sxd = reinterpret_cast<const double*>(sx);
  double out[NR];
  if (l < n) {
    const bool masked = L.ldir[l] != 0;
    const int t = threadIdx.x * NR;
    if (first) {
      const double di = 1.0 / lat_diag(L, l);
#pragma unroll
      for (int d = 0; d < NR; ++d) out[d] = (d < 2 && masked) ? 0.0 : cb * di * sbd[t + d];
    } else {
      double y[NR], diag;
      // neighbours inside the block's range come from LDS
      lat_apply<NR, M>(
          L, l,
          [&](int32_t i, int d) {
            const uint32_t r = (uint32_t)(i - l0);
            return r < (uint32_t)kBlock ? sxd[r * NR + d] : xk[(int64_t)i * NR + d];
          },
          y, diag);
      const double di = 1.0 / diag;
#pragma unroll
      for (int d = 0; d < NR; ++d) {
        const double xv = sxd[t + d];
        out[d] = (d < 2 && masked) ? 0.0 : xv + ca * (xv - smd[t + d]) + cb * di * (sbd[t + d] - y[d]);
      }
    }
  }
  __syncthreads();  // every read of sm is done: it now stages x_new
  double* smw = reinterpret_cast<double*>(sm);
  if (l < n) {
#pragma unroll
    for (int d = 0; d < NR; ++d) smw[threadIdx.x * NR + d] = out[d];
  }
  __syncthreads();
  double2* o2 = reinterpret_cast<double2*>(xnew + v0);
  double2* k2 = reinterpret_cast<double2*>(xk + v0);
#pragma unroll
  for (int q = threadIdx.x; q < kPieces; q += kBlock) {
    if (v0 + 2 * q + 1 < vend) {
      const double2 ov = sm[q];
      nt_d2 o;
      o.x = ov.x;
      o.y = ov.y;
      __builtin_nontemporal_store(o, reinterpret_cast<nt_d2*>(o2) + q);
      if (first) k2[q] = make_double2(0.0, 0.0);
    } else if (v0 + 2 * q < vend) {
      xnew[v0 + 2 * q] = smw[2 * q];
      if (first) xk[v0 + 2 * q] = 0.0;
    }
  }
}

}  // namespace

int cheb_iterations(double tol) {
  // error reduction 2 ((sqrt(k)-1)/(sqrt(k)+1))^m with k = 4 (interval [1/2, 2]),
  // times sqrt(k) from the energy norm to the scaled residual
  const double rate = 1.0 / 3.0;
  int m = (int)std::ceil(std::log(4.0 / tol) / std::log(1.0 / rate));
  return m < 1 ? 1 : m;
}

double* launch_cheb(const LatDev& L, int32_t n, const double* b, int nr,
                    double* const x[3], int iters, hipStream_t s, hipEvent_t* (*timer)(void*),
                    void* tctx) {
  // the kernel moves its block ranges as 16-byte pieces
  const uintptr_t align = (uintptr_t)b | (uintptr_t)x[0] | (uintptr_t)x[1] | (uintptr_t)x[2];
  if ((align & 15) != 0 || !lat_dispatch(L.m, [](auto) {})) return nullptr;
  const double lo = 0.5, hi = 2.0;
  const double theta = 0.5 * (hi + lo), delta = 0.5 * (hi - lo), sigma = theta / delta;
  const int g = (n + kBlock - 1) / kBlock;
  double rho = 1.0 / sigma;
  for (int k = 0; k < iters; ++k) {
    double ca = 0.0, cb = 1.0 / theta;
    if (k > 0) {
      const double rn = 1.0 / (2.0 * sigma - rho);
      ca = rn * rho;
      cb = 2.0 * rn / delta;
      rho = rn;
    }
    double* xk = x[k % 3];
    const double* xkm = x[(k + 2) % 3];
    double* xn = x[(k + 1) % 3];
    hipEvent_t* ev = (timer && k > 0) ? timer(tctx) : nullptr;
    if (ev) (void)hipEventRecord(ev[0], s);
    lat_dispatch(L.m, [&](auto lat) {
      constexpr int M = decltype(lat)::kM;
      if (nr == 3)
        k_cheb_lattice<3, M><<<g, kBlock, 0, s>>>(L, n, b, xk, xkm, xn, ca, cb, k == 0);
      else
        k_cheb_lattice<2, M><<<g, kBlock, 0, s>>>(L, n, b, xk, xkm, xn, ca, cb, k == 0);
    });
    if (ev) (void)hipEventRecord(ev[1], s);
  }
  return x[iters % 3];
}

}  // namespace cgp
