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
template <int NR, int M>
__global__ void __launch_bounds__(kBlock)
k_cheb_lattice(LatDev L, int32_t n, const double* __restrict__ b, double* __restrict__ xk,
               const double* __restrict__ xkm, double* __restrict__ xnew, double ca, double cb,
               int first) {
  const int32_t l = blockIdx.x * kBlock + threadIdx.x;
  if (l >= n) return;
  const bool masked = L.ldir[l] != 0;
  const int64_t base = (int64_t)l * NR;
  if (first) {
    const double di = 1.0 / lat_diag(L, l);
#pragma unroll
    for (int d = 0; d < NR; ++d) {
      xnew[base + d] = (d < 2 && masked) ? 0.0 : cb * di * b[base + d];
      xk[base + d] = 0.0;
    }
    return;
  }
  double y[NR], diag;
  lat_apply<NR, M>(L, l, [&](int32_t i, int d) { return xk[(int64_t)i * NR + d]; }, y, diag);
  const double di = 1.0 / diag;
#pragma unroll
  for (int d = 0; d < NR; ++d) {
    const int64_t k = base + d;
    xnew[k] = (d < 2 && masked) ? 0.0 : xk[k] + ca * (xk[k] - xkm[k]) + cb * di * (b[k] - y[d]);
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
