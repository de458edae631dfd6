// s-step coarse Jacobi-PCG (see capcg.hpp): set-up, start, one launch per s
// iterations, and the final copy-out.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "capcg.hpp"
#include "device.hpp"

namespace cgp {
namespace {

constexpr int S = kCaS, M = kCaM, NU = kCaNU, NG = kCaNG;
constexpr int T = kCaThreads, EXT = kCaExtMax, EMAX = kCaEllMax;
constexpr int kW = T / 64;         // waves per work-group
constexpr int LDE = EXT + 1;       // LDS row stride of the basis (odd: rows in different banks)
constexpr int PER = (EXT + T - 1) / T;     // neighbourhood nodes per thread
constexpr int PERE = (EMAX + T - 1) / T;   // ELL entries per thread
constexpr int kSPW = (NG + kW - 1) / kW;   // Gram entries per wave
constexpr int kTPL = 3;                    // tiles per lane per pass over the partials

// Cross-lane sums on DPP row permutations (VALU, no LDS round trip).
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

// Sum over each row of 16 lanes: quad_perm [1,0,3,2] and [2,3,0,1] (lane xor 1,
// xor 2), then row_half_mirror (lane i <- 7 - i within eight) and row_mirror
// (i <- 15 - i).  Every lane of the row ends with the same value (each step
// adds the same two numbers, only in swapped order).
__device__ __forceinline__ double row_sum16(double v) {
  v += dpp<0xB1>(v);
  v += dpp<0x4E>(v);
  v += dpp<0x141>(v);
  v += dpp<0x140>(v);
  return v;
}

__device__ __forceinline__ double read_lane(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// Sum over the wave, in a fixed order, the same value in every lane.
__device__ __forceinline__ double wsum(double v) {
  v = row_sum16(v);
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Position of (u, v), u <= v, in the packed upper triangle of an M x M matrix.
__host__ __device__ constexpr int upk(int u, int v) { return u * M - u * (u - 1) / 2 + (v - u); }

// Sum over the work-group of NS values per thread, in a fixed order; every
// thread receives the sums.
template <int NS>
__device__ void group_sums(double (&v)[NS], double* sh /* [NS][kW] */) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    const double w = wsum(v[q]);
    if (lane == 0) sh[q * kW + wv] = w;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NS; ++q) {
    double t = 0.0;
    for (int w = 0; w < kW; ++w) t += sh[q * kW + w];
    v[q] = t;
  }
  __syncthreads();
}

// Ba = B a: the Chebyshev basis satisfies A^ T_0 = T_1 + T_0 and
// A^ T_j = T_j + (T_{j+1} + T_{j-1}) / 2, applied to the first s columns of
// the p-block and the first s-1 of the r-block (the last vector of each block
// is never multiplied: its coefficient is zero whenever B is applied).
__device__ __forceinline__ void apply_b(const double (&a)[M], double (&Ba)[M]) {
#pragma unroll
  for (int k = 0; k < M; ++k) Ba[k] = 0.0;
#pragma unroll
  for (int blk = 0; blk < 2; ++blk) {
    const int off = blk == 0 ? 0 : S + 1, nb = blk == 0 ? S + 1 : S;
#pragma unroll
    for (int j = 0; j + 1 < nb; ++j) {
      const double x = a[off + j];
      if (j == 0) {
        Ba[off] += x;
        Ba[off + 1] += x;
      } else {
        Ba[off + j] += x;
        Ba[off + j + 1] += 0.5 * x;
        Ba[off + j - 1] += 0.5 * x;
      }
    }
  }
}

// x' G y with row i of G held by lane i of each 16-lane row (zero rows on
// lanes i >= M); every lane of the work-group ends with the same value.
__device__ __forceinline__ double quad(const double (&row)[M], int r16, const double (&x)[M],
                                       const double (&y)[M]) {
  double t0 = 0.0, t1 = 0.0, t2 = 0.0;
#pragma unroll
  for (int j = 0; j < M; j += 3) {
    t0 += row[j] * y[j];
    if (j + 1 < M) t1 += row[j + 1] * y[j + 1];
    if (j + 2 < M) t2 += row[j + 2] * y[j + 2];
  }
  double xi = 0.0;
#pragma unroll
  for (int m = 0; m < M; ++m) xi = r16 == m ? x[m] : xi;
  return row_sum16(xi * ((t0 + t1) + t2));
}

__global__ void k_ca_sq(CaDev d, const int32_t* __restrict__ rowptr, const double* __restrict__ Kval) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < d.n) d.sq[g] = sqrt(Kval[rowptr[d.perm[g]]]);  // rows start with the diagonal
}

__global__ void k_ca_values(CaDev d, const double* __restrict__ Kval) {
  const int t = blockIdx.x;
  const int e0 = d.ext_off[t];
  const int rows = d.layer[t * (S + 1) + S - 1];
  const int eo = d.ell_off[t];
  for (int q = threadIdx.x; q < d.width * rows; q += blockDim.x) {
    const int r = q % rows;
    const int sl = d.ell_slot[eo + q];
    double v = 0.0;
    if (sl >= 0) v = Kval[sl] / (d.sq[d.ext[e0 + r]] * d.sq[d.ext[e0 + d.ell_col[eo + q]]]);
    d.ell_val[eo + q] = v;
  }
}

__global__ void __launch_bounds__(T)
k_ca_start(CaDev d, const int32_t* __restrict__ ecol, const double* __restrict__ eval, int w,
           const double* __restrict__ b, const double* __restrict__ x, Scal* sc) {
  __shared__ double sh[2 * kW];
  const int t = blockIdx.x;
  const int o0 = d.own_off[t], no = d.own_off[t + 1] - o0;
  const int64_t n = d.n;
  double v[2] = {0.0, 0.0};
  const int k = threadIdx.x;
  if (k < no) {
    const int g = o0 + k, e = d.perm[g];
    double kx = 0.0;
    for (int q = 0; q < w; ++q) kx += eval[q * n + e] * x[ecol[q * n + e]];
    const double be = b[e], r = be - kx, sq = d.sq[g];
    d.xh[g] = sq * x[e];
    d.r0[g] = r / sq;
    v[0] = r * r;
    v[1] = be * be;
  }
  group_sums<2>(v, sh);
  if (threadIdx.x == 0) {
    d.spart[t] = v[0];
    d.spart[d.ntiles_pad + t] = v[1];
    if (t == 0) {
      Scal& s = sc[0];
      s.rho[0] = s.rho[1] = 0.0;
      s.rho_old = s.alpha = s.omega = 1.0;
      s.bb = 0.0;
      s.rel = 0.0;
      s.done_stamp = 0;
      s.iters = 0;
      s.status = 0;
    }
  }
}

// One launch = s iterations.  Every global load the launch needs (the tile's
// ELL block, the previous basis on the neighbourhood, the Gram partials of
// all tiles) is issued up front, so the launch waits for memory about once;
// the ELL block and the basis are then staged in LDS and the matrix powers
// run from LDS only.
__global__ void __launch_bounds__(T)
k_ca_outer(CaDev d, Scal* sc, int o, double tol, int max_iter, int my_stamp) {
  __shared__ double lv[M * LDE];      // basis levels on the neighbourhood
  __shared__ double sval[EMAX];       // the tile's ELL block
  __shared__ uint16_t scol[EMAX];
  __shared__ double gs[NG];
  __shared__ double sd[T];
  __shared__ double sh[2 * kW];
  __shared__ double cf[3 * M + 1];  // a, c, e and ||r||^2 from wave 0
  __shared__ int cfi[3];            // steps taken, stop, NaN
  const int t = blockIdx.x;
  const int o0 = d.own_off[t], no = d.own_off[t + 1] - o0;
  const int e0 = d.ext_off[t], ne = d.ext_off[t + 1] - e0;
  const int32_t* lay = d.layer + t * (S + 1);
  const int rows = lay[S - 1];
  const int eo = d.ell_off[t], wd = d.width, nent = wd * rows;
  const int64_t n = d.n;
  const int par = o & 1, prev = par ^ 1;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;

  // (1) loads: ELL block, basis (or r^_0) at the neighbourhood, partials
  double ev[PERE];
  int ec[PERE];
#pragma unroll
  for (int u = 0; u < PERE; ++u) {
    const int q = tid + u * T;
    ev[u] = 0.0;
    ec[u] = 0;
    if (q < nent) {
      ev[u] = d.ell_val[eo + q];
      ec[u] = d.ell_col[eo + q];
    }
  }
  double vv[PER][M];
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int r = tid + q * T;
#pragma unroll
    for (int m = 0; m < M; ++m) vv[q][m] = 0.0;
    if (r < ne) {
      const int g = d.ext[e0 + r];
      if (o == 1) {
        vv[q][0] = d.r0[g];
      } else {
#pragma unroll
        for (int m = 0; m < M; ++m) vv[q][m] = d.V[prev][m * n + g];
      }
    }
  }
  // Gram partials: wave wv sums entries wv, wv + kW, ...; lane takes tiles
  // lane, lane + 64, ... (first kTPL * 64 tiles here, any others below)
  double pv[kSPW][kTPL];
  if (o >= 2) {
#pragma unroll
    for (int i = 0; i < kSPW; ++i) {
      const int kk = wv + kW * i;
      const double* src = d.gpart + ((int64_t)prev * NG + (kk < NG ? kk : 0)) * d.ntiles_pad;
#pragma unroll
      for (int u = 0; u < kTPL; ++u) {
        const int tt = lane + 64 * u;
        pv[i][u] = (kk < NG && tt < d.ntiles) ? src[tt] : 0.0;
      }
    }
  }
  const int stamp0 = sc[0].done_stamp;
  const double bb_prev = sc[0].bb;

  // (2) stage the ELL block and the basis
#pragma unroll
  for (int u = 0; u < PERE; ++u) {
    const int q = tid + u * T;
    if (q < nent) {
      sval[q] = ev[u];
      scol[q] = (uint16_t)ec[u];
    }
  }
#pragma unroll
  for (int q = 0; q < PER; ++q) {
    const int r = tid + q * T;
    if (r < ne) {
      if (o == 1) {
        lv[r] = vv[q][0];  // p^ = r^ = r^_0
        if (r < rows) lv[(S + 1) * LDE + r] = vv[q][0];
      } else {
#pragma unroll
        for (int m = 0; m < M; ++m) lv[m * LDE + r] = vv[q][m];
      }
    }
  }
  if (!(stamp0 == 0 || stamp0 >= my_stamp)) return;  // solve already finished

  if (o == 1) {
    // test of the guess
    double v[2] = {0.0, 0.0};
    for (int tt = tid; tt < d.ntiles; tt += T) {
      v[0] += d.spart[tt];
      v[1] += d.spart[d.ntiles_pad + tt];
    }
    group_sums<2>(v, sh);
    const double rr = v[0], bb = v[1];
    const double rel = bb > 0.0 ? sqrt(rr / bb) : 0.0;
    const bool nan = !isfinite(bb) || !isfinite(rr) || !isfinite(rel);
    const bool fin = bb == 0.0 || nan || rel <= tol;
    if (t == 0 && tid == 0) {
      sc[0].bb = bb;
      sc[0].rel = rel;
      if (fin) {
        sc[0].done_stamp = my_stamp;
        sc[0].iters = 0;
        sc[0].status = nan ? 2 : 0;
      }
    }
    if (bb == 0.0) {  // zero right-hand side: the solution is zero
      if (tid < no) d.xh[o0 + tid] = 0.0;
      return;
    }
    if (fin) return;
  } else {
    // (3) Gram matrices of the previous basis, summed over tiles in a fixed order
    double gacc[kSPW];
#pragma unroll
    for (int i = 0; i < kSPW; ++i) {
      gacc[i] = 0.0;
#pragma unroll
      for (int u = 0; u < kTPL; ++u) gacc[i] += pv[i][u];
    }
    for (int t0 = 64 * kTPL; t0 < d.ntiles; t0 += 64 * kTPL) {
#pragma unroll
      for (int i = 0; i < kSPW; ++i) {
        const int kk = wv + kW * i;
        const double* src = d.gpart + ((int64_t)prev * NG + (kk < NG ? kk : 0)) * d.ntiles_pad;
#pragma unroll
        for (int u = 0; u < kTPL; ++u) {
          const int tt = t0 + lane + 64 * u;
          gacc[i] += (kk < NG && tt < d.ntiles) ? src[tt] : 0.0;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kSPW; ++i) {
      const double a = wsum(gacc[i]);
      const int kk = wv + kW * i;
      if (lane == 0 && kk < NG) gs[kk] = a;
    }
    __syncthreads();
    // (4) the s CG steps on coefficient vectors, on wave 0 (the others wait;
    // a wave64 FP64 instruction holds its SIMD for four cycles, so the serial
    // steps are run once), results through LDS
    const int it0 = (o - 2) * S;
    const int nin = min(S, max_iter - it0);
    if (wv == 0) {
      const int r16 = lane & 15;
      double grow[M], gdrow[M];
#pragma unroll
      for (int j = 0; j < M; ++j) {
        const int pk = r16 <= j ? upk(r16, j) : upk(j, r16);
        grow[j] = r16 < M ? gs[pk] : 0.0;
        gdrow[j] = r16 < M ? gs[NU + pk] : 0.0;
      }
      // row r16 of G B, so that p'A^p = a'G(Ba) is a quadratic form in a
      // alone and B a leaves the critical path
      double gbrow[M];
#pragma unroll
      for (int blk = 0; blk < 2; ++blk) {
        const int off = blk == 0 ? 0 : S + 1, nb = blk == 0 ? S + 1 : S;
#pragma unroll
        for (int jj = 0; jj < nb; ++jj) {
          const int J = off + jj;
          double v = 0.0;
          if (jj + 1 < nb) {
            v = jj == 0 ? grow[off] + grow[off + 1]
                        : grow[J] + 0.5 * (grow[J + 1] + grow[J - 1]);
          }
          gbrow[J] = v;
        }
      }
      double a[M], c[M], e[M];
#pragma unroll
      for (int m = 0; m < M; ++m) a[m] = c[m] = e[m] = 0.0;
      a[0] = 1.0;
      c[S + 1] = 1.0;
      double rz = quad(grow, r16, c, c);
      bool fin = false, nan = false;
      double rr = 0.0;
      const double tol2bb = tol * tol * bb_prev;  // ||r|| <= tol ||b||
      // the four steps unrolled (guarded by the step budget and the stop), so
      // that the entries of a, c, e still zero at each step fold away
      int j = 0;
#pragma unroll
      for (int jj = 0; jj < S; ++jj) {
        if (jj < nin && !fin) {
          const double den = quad(gbrow, r16, a, a);
          double Ba[M];
          apply_b(a, Ba);
          const double inv_rz = 1.0 / rz;
          const double al = rz / den;
#pragma unroll
          for (int m = 0; m < M; ++m) {
            e[m] += al * a[m];
            c[m] -= al * Ba[m];
          }
          j = jj + 1;
          rr = quad(gdrow, r16, c, c);
          const double rzn = quad(grow, r16, c, c);
          nan = !isfinite(rr) || !isfinite(al);
          if (nan || fabs(rr) <= tol2bb) {
            fin = true;
          } else {
            const double be = rzn * inv_rz;
            rz = rzn;
#pragma unroll
            for (int m = 0; m < M; ++m) a[m] = c[m] + be * a[m];
          }
        }
      }
      if (lane == 0) {
#pragma unroll
        for (int m = 0; m < M; ++m) {
          cf[m] = a[m];
          cf[M + m] = c[m];
          cf[2 * M + m] = e[m];
        }
        cf[3 * M] = rr;
        cfi[0] = j;
        cfi[1] = fin ? 1 : 0;
        cfi[2] = nan ? 1 : 0;
      }
    }
    __syncthreads();
    double a[M], c[M], e[M];
#pragma unroll
    for (int m = 0; m < M; ++m) {
      a[m] = cf[m];
      c[m] = cf[M + m];
      e[m] = cf[2 * M + m];
    }
    const double rr = cf[3 * M];
    const int j = cfi[0];
    const bool fin = cfi[1] != 0, nan = cfi[2] != 0;
    if (t == 0 && tid == 0) {
      sc[0].rel = bb_prev > 0.0 ? sqrt(fabs(rr) / bb_prev) : 0.0;
      if (fin) {
        sc[0].done_stamp = my_stamp;
        sc[0].iters = it0 + j;
        sc[0].status = nan ? 2 : 0;
      }
    }
    // (5) x^ at the own nodes, and p^, r^ on the neighbourhood (in place:
    // each thread reads and rewrites only its own columns of lv)
    const bool last = fin || it0 + nin >= max_iter;
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int r = tid + q * T;
      if (r < ne) {
        double vals[M];
#pragma unroll
        for (int m = 0; m < M; ++m) vals[m] = lv[m * LDE + r];
        if (q == 0 && r < no && !nan) {
          double dx = 0.0;
#pragma unroll
          for (int m = 0; m < M; ++m) dx += vals[m] * e[m];
          d.xh[o0 + r] += dx;
        }
        if (!last) {
          double pv2 = 0.0, rv2 = 0.0;
#pragma unroll
          for (int m = 0; m < M; ++m) {
            pv2 += vals[m] * a[m];
            rv2 += vals[m] * c[m];
          }
          lv[r] = pv2;
          if (r < rows) lv[(S + 1) * LDE + r] = rv2;
        }
      }
    }
    if (last) return;
  }
  if (tid < no) {
    const double q = d.sq[o0 + tid];
    sd[tid] = q * q;
  }
  __syncthreads();

  // (6) matrix powers from LDS: level j of the p-block on distance <= s - j,
  // of the r-block on distance <= s - 1 - j
  // the first 8 entries of the thread's rows tid and tid + T, held in
  // registers over all passes (rows <= EXT = 2 T)
  int rc[2][8];
  double rv[2][8];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int r = tid + h * T;
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const bool ok = r < rows && u < wd;
      rc[h][u] = ok ? scol[u * rows + r] : 0;
      rv[h][u] = ok ? sval[u * rows + r] : 0.0;
    }
  }
  for (int j = 1; j <= S; ++j) {
#pragma unroll
    for (int blk = 0; blk < 2; ++blk) {
      if (blk == 1 && j > S - 1) continue;
      const int base = blk == 0 ? 0 : S + 1;
      const int nrow = blk == 0 ? lay[S - j] : lay[S - 1 - j];
      const double* src = lv + (base + j - 1) * LDE;
      const double* src2 = lv + (base + (j >= 2 ? j - 2 : 0)) * LDE;  // read only for j >= 2
      double* dst = lv + (base + j) * LDE;
      {
        const int r0 = tid;
        double y[2] = {0.0, 0.0};
        {
          double xs[2][8];
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int u = 0; u < 8; ++u) xs[h][u] = src[rc[h][u]];
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int u = 0; u < 8; ++u) y[h] += rv[h][u] * xs[h][u];
        }
        // entries beyond the first 8 (wider rows), per batch of 8
        for (int k0 = 8; k0 < wd; k0 += 8) {
          int cc[2][8];
          double va[2][8], xs[2][8];
#pragma unroll
          for (int h = 0; h < 2; ++h) {
            const int r = r0 + h * T;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
              const bool ok = r < nrow && k0 + u < wd;
              const int at = (k0 + u) * rows + r;
              cc[h][u] = ok ? scol[at] : 0;
              va[h][u] = ok ? sval[at] : 0.0;
            }
          }
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int u = 0; u < 8; ++u) xs[h][u] = src[cc[h][u]];
#pragma unroll
          for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int u = 0; u < 8; ++u) y[h] += va[h][u] * xs[h][u];
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int r = r0 + h * T;
          if (r < nrow) dst[r] = j == 1 ? y[h] - src[r] : 2.0 * (y[h] - src[r]) - src2[r];
        }
      }
    }
    __syncthreads();
  }

  // (7) the new basis at the own nodes, and its Gram partials.  The 9 x 9
  // matrices are cut into 3 x 3 blocks; wave w < 6 takes block (bu, bv),
  // bu <= bv, each lane accumulates G and G_D over own nodes lane, lane + 64,
  // ... in registers, and every entry is summed over the wave by one butterfly
  // in a fixed order.
  if (tid < no) {
#pragma unroll
    for (int m = 0; m < M; ++m) d.V[par][m * n + o0 + tid] = lv[m * LDE + tid];
  }
  if (wv < 6) {
    const int bu = wv < 3 ? 0 : (wv < 5 ? 1 : 2);
    const int bv = wv < 3 ? wv : (wv < 5 ? wv - 2 : 2);
    double ag[3][3], ad[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) ag[i][j] = ad[i][j] = 0.0;
    // every own node slot of the lane (at most T / 64), all reads issued together
#pragma unroll
    for (int q = 0; q < T / 64; ++q) {
      const int k = lane + 64 * q;
      if (k >= no) continue;
      double xu[3], xw[3];
      const double dk = sd[k];
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        xu[i] = lv[(3 * bu + i) * LDE + k];
        xw[i] = lv[(3 * bv + i) * LDE + k];
      }
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          const double pr = xu[i] * xw[j];
          ag[i][j] += pr;
          ad[i][j] += dk * pr;
        }
    }
    double* gp = d.gpart + (int64_t)par * NG * d.ntiles_pad + t;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        if (bu == bv && i > j) continue;  // lower half of a diagonal block
        const double g = wsum(ag[i][j]), gd = wsum(ad[i][j]);
        if (lane == 0) {
          const int pk = upk(3 * bu + i, 3 * bv + j);
          gp[(int64_t)pk * d.ntiles_pad] = g;
          gp[(int64_t)(NU + pk) * d.ntiles_pad] = gd;
        }
      }
  }
}

__global__ void k_ca_final(CaDev d, double* __restrict__ x) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < d.n) x[d.perm[g]] = d.xh[g] / d.sq[g];
}

}  // namespace

static_assert(kCaM == 9 && kCaThreads >= 6 * 64, "Gram partials: six waves, 3 x 3 blocks");
static_assert(kCaExtMax <= 65535, "local column indices are 16-bit");
static_assert(kCaExtMax <= 2 * kCaThreads, "the matrix powers give each thread at most two rows");

void launch_ca_setup(const CaDev& d, const int32_t* rowptr, const double* Kval, hipStream_t s) {
  k_ca_sq<<<(d.n + 255) / 256, 256, 0, s>>>(d, rowptr, Kval);
  k_ca_values<<<d.ntiles, 256, 0, s>>>(d, Kval);
}

void launch_ca_start(const CaDev& d, const int32_t* ell_col, const double* ell_val, int ell_w,
                     const double* b, const double* x, Scal* sc, hipStream_t s) {
  k_ca_start<<<d.ntiles, T, 0, s>>>(d, ell_col, ell_val, ell_w, b, x, sc);
}

void launch_ca_outer(const CaDev& d, Scal* sc, int o, double tol, int max_iter, int my_stamp,
                     hipStream_t s, hipEvent_t* ev) {
  if (ev) (void)hipEventRecord(ev[0], s);
  k_ca_outer<<<d.ntiles, T, 0, s>>>(d, sc, o, tol, max_iter, my_stamp);
  if (ev) (void)hipEventRecord(ev[1], s);
}

void launch_ca_final(const CaDev& d, double* x, hipStream_t s) {
  k_ca_final<<<(d.n + 255) / 256, 256, 0, s>>>(d, x);
}

}  // namespace cgp
