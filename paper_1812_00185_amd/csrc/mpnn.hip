// Learned initial guess for the coarse Poisson solve: a 3-round
// message-passing network (hidden width 32) on the coarse node graph,
// forward, backward and Adam, for gfx950.
//
// Network (per node i, edges = off-diagonal CSR slots of the coarse graph):
//   q = 3 phi^n - 3 phi^{n-1} + phi^{n-2} (quadratic extrapolation in time),
//   e = phi^n - 3 phi^{n-1} + 3 phi^{n-2} - phi^{n-3} (its last error),
//   x_i = [b_i/s_b, (b - K q)_i/s, e_i/s, d1_i/s_1, d2_i/s_2], s ~ rms(e),
//   d1, d2 the first and second differences of the history
//   h = relu(W_e x + c_e)
//   round r: p = A_r h, q = B_r h, m_ij = relu(p_i + q_j + C_r e_ij + d_r),
//            a_i = mean_j m_ij, h <- h + relu(U_r [h; a] + v_r)
//   y = w . h + c,  guess = q + s y
// Dense layers run on BF16 MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulate);
// since the message is linear before its activation, the only dense
// products are per node (p, q together as one 32 -> 64 layer; the update as
// one 64 -> 32 layer) and the edge stage is elementwise.  Weight gradients
// are MFMA products over rows, summed per block and reduced in a fixed order;
// gradients that gather over edges use the symmetric graph instead of
// atomics, so training is bitwise reproducible.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "device.hpp"
#include "mpnn.hpp"

namespace cgp {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kB = 256;  // threads per block (4 waves)

__device__ __forceinline__ float wave_sumf(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_sumd(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// ---------------------------------------------------------------- dense layers
// Y[M][N] = act(X Wt + bias) (+ residual), X = [X1 | X2] with K1 + K2 columns,
// W stored BF16 row-major [N][K] (output x input).  One wave computes 16 rows
// x N; MFMA 16x16x32 lane layout: A row = lane % 16, k = 8 (lane / 16) + e;
// B column = lane % 16, k = 8 (lane / 16) + e; D column = lane % 16,
// row = 4 (lane / 16) + e.
// MODE 0: Y = XW^T (+bias); MODE 1: Z = XW^T + bias stored, Y = relu(Z);
// MODE 2: Z stored, Y = resid + relu(Z).
template <int K1, int K2, int N, int MODE>
__global__ void __launch_bounds__(kB)
k_dense(int M, const float* __restrict__ X1, const float* __restrict__ X2,
        const __bf16* __restrict__ W, const float* __restrict__ bias,
        const float* __restrict__ resid, float* __restrict__ Z, float* __restrict__ Y) {
  constexpr int K = K1 + K2;
  static_assert(K % 32 == 0 && N % 16 == 0, "MFMA tile shape");
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int row0 = (blockIdx.x * (kB / 64) + wave) * 16;
  if (row0 >= M) return;  // whole wave
  const int lr = lane & 15, kg = lane >> 4;
  const int row = row0 + lr;
  bf16x8 a[K / 32];
#pragma unroll
  for (int ks = 0; ks < K / 32; ++ks)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int k = ks * 32 + kg * 8 + e;
      float v = 0.0f;
      if (row < M) v = k < K1 ? X1[(int64_t)row * K1 + k] : X2[(int64_t)row * K2 + (k - K1)];
      a[ks][e] = (__bf16)v;
    }
#pragma unroll
  for (int nt = 0; nt < N / 16; ++nt) {
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    const int n = nt * 16 + lr;
#pragma unroll
    for (int ks = 0; ks < K / 32; ++ks) {
      bf16x8 b;
#pragma unroll
      for (int e = 0; e < 8; ++e) b[e] = W[n * K + ks * 32 + kg * 8 + e];
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[ks], b, acc, 0, 0, 0);
    }
    const float bn = bias ? bias[n] : 0.0f;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int r = row0 + kg * 4 + e;
      if (r >= M) continue;
      const float z = acc[e] + bn;
      const int64_t o = (int64_t)r * N + n;
      if (MODE == 0) {
        Y[o] = z;
      } else if (MODE == 1) {
        Z[o] = z;
        Y[o] = fmaxf(z, 0.0f);
      } else {
        Z[o] = z;
        Y[o] = resid[o] + fmaxf(z, 0.0f);
      }
    }
  }
}

// Weight gradient partials: G[n][k] = sum over this block's rows of
// dY[r][n] X[r][k] (MFMA with the rows as the reduction dimension), and the
// bias gradient sum_r dY[r][n].  part: [block][NOUT * K + NOUT].
template <int K1, int K2, int NOUT>
__global__ void __launch_bounds__(kB)
k_wgrad(int M, int rows_per_block, const float* __restrict__ dY, const float* __restrict__ X1,
        const float* __restrict__ X2, float* __restrict__ part) {
  constexpr int K = K1 + K2;
  constexpr int TN = NOUT / 16, TK = K / 16;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int lr = lane & 15, kg = lane >> 4;
  const int rb = blockIdx.x * rows_per_block;
  const int re = min(M, rb + rows_per_block);
  float* out = part + (int64_t)blockIdx.x * (NOUT * K + NOUT);
  for (int t = wave; t < TN * TK; t += kB / 64) {
    const int tn = t / TK, tk = t % TK;
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
    const int n = tn * 16 + lr, k = tk * 16 + lr;
    for (int r0 = rb; r0 < re; r0 += 32) {
      bf16x8 a, b;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int r = r0 + kg * 8 + e;
        const bool ok = r < re;
        a[e] = (__bf16)(ok ? dY[(int64_t)r * NOUT + n] : 0.0f);
        float xv = 0.0f;
        if (ok) xv = k < K1 ? X1[(int64_t)r * K1 + k] : X2[(int64_t)r * K2 + (k - K1)];
        b[e] = (__bf16)xv;
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int e = 0; e < 4; ++e) out[(tn * 16 + kg * 4 + e) * K + tk * 16 + lr] = acc[e];
  }
  // bias gradient: NG row groups of NOUT columns, reduced through LDS
  constexpr int NG = kB / NOUT;
  __shared__ float sb[NG][NOUT];
  {
    const int col = threadIdx.x % NOUT, grp = threadIdx.x / NOUT;
    float s = 0.0f;
    for (int r = rb + grp; r < re; r += NG) s += dY[(int64_t)r * NOUT + col];
    sb[grp][col] = s;
  }
  __syncthreads();
  if (threadIdx.x < NOUT) {
    float s = 0.0f;
    for (int g = 0; g < NG; ++g) s += sb[g][threadIdx.x];
    out[NOUT * K + threadIdx.x] = s;
  }
}

// Sums the per-block partials in block order into grad: weights of shape
// [NOUT][KREAL] (the first KREAL of K columns) at wofs, biases at bofs (< 0:
// none).
__global__ void k_wgrad_reduce(const float* __restrict__ part, int nblk, int nout, int k,
                               int kreal, float* __restrict__ grad, int wofs, int bofs) {
  const int per = nout * k + nout;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < per; i += gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * per + i];
    if (i < nout * k) {
      const int n = i / k, kk = i % k;
      if (kk < kreal) grad[wofs + n * kreal + kk] = s;
    } else if (bofs >= 0) {
      grad[bofs + (i - nout * k)] = s;
    }
  }
}

// ---------------------------------------------------------------- graph stages
// Edge features of every off-diagonal slot: ((x_j - x_i)/hbar, (y_j - y_i)/hbar, len/hbar, 0)
__global__ void k_edge_features(DLevel C, float hbar_inv, float4* __restrict__ ef,
                                float* __restrict__ deg_inv) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < C.n; i += gridDim.x * blockDim.x) {
    const int beg = C.rowptr[i], end = C.rowptr[i + 1];
    const double2 pi = C.xy[i];
    for (int s = beg + 1; s < end; ++s) {
      const double2 pj = C.xy[C.col[s]];
      const double dx = pj.x - pi.x, dy = pj.y - pi.y;
      ef[s] = make_float4((float)(dx * hbar_inv), (float)(dy * hbar_inv),
                          (float)(sqrt(dx * dx + dy * dy) * hbar_inv), 0.0f);
    }
    ef[beg] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    deg_inv[i] = end - beg > 1 ? 1.0f / (float)(end - beg - 1) : 0.0f;
  }
}

// a_i = deg_inv_i sum_j relu(p_i + q_j + C e_ij + d); 32 lanes (channels) per node.
__global__ void __launch_bounds__(kB)
k_edge_fwd(DLevel C, const float4* __restrict__ ef, const float* __restrict__ deg_inv,
           const float* __restrict__ PQ, const float* __restrict__ Cw, const float* __restrict__ d,
           float* __restrict__ A) {
  const int c = threadIdx.x & 31;
  const int i = blockIdx.x * (kB / 32) + (threadIdx.x >> 5);
  if (i >= C.n) return;
  const float p = PQ[(int64_t)i * 64 + c];
  const float c0 = Cw[c * 3], c1 = Cw[c * 3 + 1], c2 = Cw[c * 3 + 2], dc = d[c];
  float acc = 0.0f;
  for (int s = C.rowptr[i] + 1; s < C.rowptr[i + 1]; ++s) {
    const int j = C.col[s];
    const float4 e = ef[s];
    const float z = p + PQ[(int64_t)j * 64 + 32 + c] + c0 * e.x + c1 * e.y + c2 * e.z + dc;
    acc += fmaxf(z, 0.0f);
  }
  A[(int64_t)i * 32 + c] = acc * deg_inv[i];
}

// Backward of the edge stage.  dS_ij = (dA_i deg_inv_i) [s_ij > 0];
// dP_i = sum_j dS_ij; dQ_i = sum_j dS_ji (reverse edges, recomputed from the
// symmetric graph: e_ji = (-e_ij.x, -e_ij.y, e_ij.len)); per-block partials
// of dC = sum dS_ij e_ij^T and dd = sum dS_ij over the block's source nodes.
__global__ void __launch_bounds__(kB)
k_edge_bwd(DLevel C, const float4* __restrict__ ef, const float* __restrict__ deg_inv,
           const float* __restrict__ PQ, const float* __restrict__ Cw, const float* __restrict__ d,
           const float* __restrict__ dA, float* __restrict__ dPQ, float* __restrict__ part) {
  __shared__ float sh[kB / 32][32][4];
  const int c = threadIdx.x & 31, slot = threadIdx.x >> 5;
  const int i = blockIdx.x * (kB / 32) + slot;
  float g0 = 0.0f, g1 = 0.0f, g2 = 0.0f, gd = 0.0f;
  if (i < C.n) {
    const float pi = PQ[(int64_t)i * 64 + c], qi = PQ[(int64_t)i * 64 + 32 + c];
    const float c0 = Cw[c * 3], c1 = Cw[c * 3 + 1], c2 = Cw[c * 3 + 2], dc = d[c];
    const float gi = dA[(int64_t)i * 32 + c] * deg_inv[i];
    float dp = 0.0f, dq = 0.0f;
    for (int s = C.rowptr[i] + 1; s < C.rowptr[i + 1]; ++s) {
      const int j = C.col[s];
      const float4 e = ef[s];
      const float pj = PQ[(int64_t)j * 64 + c], qj = PQ[(int64_t)j * 64 + 32 + c];
      // edge i -> j
      const float sij = pi + qj + c0 * e.x + c1 * e.y + c2 * e.z + dc;
      const float dsij = sij > 0.0f ? gi : 0.0f;
      dp += dsij;
      g0 += dsij * e.x;
      g1 += dsij * e.y;
      g2 += dsij * e.z;
      gd += dsij;
      // edge j -> i
      const float sji = pj + qi - c0 * e.x - c1 * e.y + c2 * e.z + dc;
      if (sji > 0.0f) dq += dA[(int64_t)j * 32 + c] * deg_inv[j];
    }
    dPQ[(int64_t)i * 64 + c] = dp;
    dPQ[(int64_t)i * 64 + 32 + c] = dq;
  }
  sh[slot][c][0] = g0;
  sh[slot][c][1] = g1;
  sh[slot][c][2] = g2;
  sh[slot][c][3] = gd;
  __syncthreads();
  if (threadIdx.x < 128) {
    const int cc = threadIdx.x >> 2, q = threadIdx.x & 3;
    float s = 0.0f;
    for (int k = 0; k < kB / 32; ++k) s += sh[k][cc][q];
    part[(int64_t)blockIdx.x * 128 + cc * 4 + q] = s;
  }
}

// dC (32 x 3) and dd (32) from the per-block partials, in block order.
__global__ void k_edge_grad_reduce(const float* __restrict__ part, int nblk,
                                   float* __restrict__ grad, int cofs, int dofs) {
  const int t = threadIdx.x;
  if (t >= 128) return;
  float s = 0.0f;
  for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * 128 + t];
  const int cc = t >> 2, q = t & 3;
  if (q < 3)
    grad[cofs + cc * 3 + q] = s;
  else
    grad[dofs + cc] = s;
}

// ---------------------------------------------------------------- features, decoder, loss
// The network-free quadratic extrapolation of the history that the network
// refines, q = 3 phi^n - 3 phi^{n-1} + phi^{n-2}, zero at the phi = 0 nodes.
__global__ void __launch_bounds__(kB)
k_extrapolate(int n, const double* __restrict__ h0, const double* __restrict__ h1,
              const double* __restrict__ h2, const uint8_t* __restrict__ nat,
              double* __restrict__ q) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
    q[i] = (nat && nat[i]) ? 0.0 : 3.0 * h0[i] - 3.0 * h1[i] + h2[i];
}

// Per-block partial sums (double) of b^2, e^2, (phi^n)^2, d1^2, d2^2 with
// e = phi^n - 3 phi^{n-1} + 3 phi^{n-2} - phi^{n-3}, d1 = phi^n - phi^{n-1},
// d2 = phi^n - 2 phi^{n-1} + phi^{n-2}.
constexpr int kStats = 5;
__global__ void __launch_bounds__(kB)
k_net_stats(int n, const double* __restrict__ b, const double* __restrict__ h0,
            const double* __restrict__ h1, const double* __restrict__ h2,
            const double* __restrict__ h3, double* __restrict__ part) {
  __shared__ double sh[kStats][kB / 64];
  double acc[kStats] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double p0 = h0[i], p1 = h1[i], p2 = h2[i], p3 = h3[i];
    const double e = p0 - 3.0 * p1 + 3.0 * p2 - p3;
    const double d1 = p0 - p1, d2 = p0 - 2.0 * p1 + p2;
    acc[0] += b[i] * b[i];
    acc[1] += e * e;
    acc[2] += p0 * p0;
    acc[3] += d1 * d1;
    acc[4] += d2 * d2;
  }
#pragma unroll
  for (int k = 0; k < kStats; ++k) {
    const double v = wave_sumd(acc[k]);
    if ((threadIdx.x & 63) == 0) sh[k][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < kStats) {
    double a = 0.0;
    for (int w = 0; w < kB / 64; ++w) a += sh[threadIdx.x][w];
    part[kStats * blockIdx.x + threadIdx.x] = a;
  }
}

// Scales (every block sums the partials in order), the quadratic
// extrapolation q = 3 phi^n - 3 phi^{n-1} + phi^{n-2} and the padded inputs
// Xf[i][0..31] = [b/s_b, (b - K q)/s, e/s, d1/s_1, d2/s_2, 0...] with
// s = max(rms(e), 1e-12 rms(phi^n)), else s_b / hbar^2 (the coarse solution
// scales like b / h^2), s_k = rms(d_k) (1 if zero); K is the solver's coarse
// operator.  Block 0 stores (s_b, s, s_1, s_2) in scal[0..3].
__global__ void __launch_bounds__(kB)
k_net_features(DLevel C, const double* __restrict__ K, const double* __restrict__ part,
               int nblk, double hbar, const double* __restrict__ b,
               const double* __restrict__ h0, const double* __restrict__ h1,
               const double* __restrict__ h2, const double* __restrict__ h3,
               float* __restrict__ Xf, double* __restrict__ qout, double* __restrict__ scal) {
  const int n = C.n;
  double t[kStats] = {0.0, 0.0, 0.0, 0.0, 0.0};
  for (int k = 0; k < nblk; ++k)
#pragma unroll
    for (int j = 0; j < kStats; ++j) t[j] += part[kStats * k + j];
  double sb = sqrt(t[0] / n);
  if (!(sb > 0.0)) sb = 1.0;
  double s = fmax(sqrt(t[1] / n), 1e-12 * sqrt(t[2] / n));
  if (!(s > 0.0)) s = sb / (hbar * hbar);
  double s1 = sqrt(t[3] / n), s2 = sqrt(t[4] / n);
  if (!(s1 > 0.0)) s1 = 1.0;
  if (!(s2 > 0.0)) s2 = 1.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    scal[0] = sb;
    scal[1] = s;
    scal[2] = s1;
    scal[3] = s2;
  }
  const double isb = 1.0 / sb, is = 1.0 / s, is1 = 1.0 / s1, is2 = 1.0 / s2;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    double kq = 0.0;
    for (int r = C.rowptr[i]; r < C.rowptr[i + 1]; ++r) {
      const int j = C.col[r];
      kq += K[r] * (3.0 * h0[j] - 3.0 * h1[j] + h2[j]);
    }
    const double p0 = h0[i], p1 = h1[i], p2 = h2[i];
    const double q = 3.0 * p0 - 3.0 * p1 + p2;
    qout[i] = q;
    float* x = Xf + (int64_t)i * 32;
    x[0] = (float)(b[i] * isb);
    x[1] = (float)((b[i] - kq) * is);
    x[2] = (float)((p0 - 3.0 * p1 + 3.0 * p2 - h3[i]) * is);
    x[3] = (float)((p0 - p1) * is1);
    x[4] = (float)((p0 - 2.0 * p1 + p2) * is2);
#pragma unroll
    for (int k = 5; k < 32; ++k) x[k] = 0.0f;
  }
}

// Per-block partial sums of t_i^2, t_i = (phi_t - q_i)/s, into tpart.
__global__ void __launch_bounds__(kB)
k_target_sq(int n, const double* __restrict__ q, const double* __restrict__ scal,
            const double* __restrict__ target, double* __restrict__ tpart) {
  __shared__ double sh[kB / 64];
  const double is = 1.0 / scal[1];
  double acc = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const double t = (target[i] - q[i]) * is;
    acc += t * t;
  }
  acc = wave_sumd(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int k = 0; k < kB / 64; ++k) a += sh[k];
    tpart[blockIdx.x] = a;
  }
}

// y_i = w . h_i + c.  With a target: t_i = (phi_t - q_i)/s, the sample weight
// 1 / max(1, mean t^2) (from the nblk partials in tpart, summed in order by
// every block), dy_i = 2 wgt (y_i - t_i) / n and per-block partials of
// wgt (y_i - t_i)^2 in lpart.  Without: guess_i = q_i + s y_i.
__global__ void __launch_bounds__(kB)
k_decoder(int n, const float* __restrict__ Hf, const float* __restrict__ w, const float* __restrict__ c,
          const double* __restrict__ scal, const double* __restrict__ q,
          const double* __restrict__ target, const double* __restrict__ tpart, int nblk,
          float* __restrict__ dy, double* __restrict__ guess, const uint8_t* __restrict__ nat,
          double* __restrict__ lpart) {
  __shared__ double sh[kB / 64];
  const double s = scal[1];
  double wgt = 1.0;
  if (target) {
    double tt = 0.0;
    for (int k = 0; k < nblk; ++k) tt += tpart[k];
    wgt = 1.0 / fmax(1.0, tt / n);
  }
  double lsum = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float* h = Hf + (int64_t)i * 32;
    float y = c[0];
#pragma unroll
    for (int k = 0; k < 32; ++k) y += w[k] * h[k];
    if (target) {
      const double t = (target[i] - q[i]) / s;
      const double r = (double)y - t;
      lsum += r * r;
      dy[i] = (float)(2.0 * wgt * r / n);
    } else {
      guess[i] = (nat && nat[i]) ? 0.0 : q[i] + s * (double)y;
    }
  }
  if (!target) return;
  lsum = wave_sumd(lsum);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = lsum;
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = 0.0;
    for (int k = 0; k < kB / 64; ++k) a += sh[k];
    lpart[blockIdx.x] = wgt * a;
  }
}

// decoder backward: dH[i][k] = dy_i w_k; partial sums of dy_i h_i (32) and dy_i
__global__ void __launch_bounds__(kB)
k_decoder_bwd(int n, const float* __restrict__ Hf, const float* __restrict__ w,
              const float* __restrict__ dy, float* __restrict__ dH, float* __restrict__ part) {
  __shared__ float sh[kB / 32][33];
  const int c = threadIdx.x & 31, slot = threadIdx.x >> 5;
  float gw = 0.0f, gc = 0.0f;
  for (int i = blockIdx.x * (kB / 32) + slot; i < n; i += gridDim.x * (kB / 32)) {
    const float g = dy[i];
    dH[(int64_t)i * 32 + c] = g * w[c];
    gw += g * Hf[(int64_t)i * 32 + c];
    gc += g;
  }
  sh[slot][c] = gw;
  if (c == 0) sh[slot][32] = gc;
  __syncthreads();
  if (threadIdx.x < 33) {
    float s = 0.0f;
    for (int k = 0; k < kB / 32; ++k) s += sh[k][threadIdx.x];
    part[(int64_t)blockIdx.x * 33 + threadIdx.x] = s;
  }
}

__global__ void k_decoder_grad_reduce(const float* __restrict__ part, int nblk, float* grad,
                                      int wofs, int cofs, const double* __restrict__ lpart,
                                      int nlblk, int n, float* loss) {
  const int t = threadIdx.x;
  if (t < 33) {
    float s = 0.0f;
    for (int b = 0; b < nblk; ++b) s += part[(int64_t)b * 33 + t];
    if (t < 32)
      grad[wofs + t] = s;
    else
      grad[cofs] = s;
  }
  if (t == 64 && loss) {
    double a = 0.0;
    for (int b = 0; b < nlblk; ++b) a += lpart[b];
    loss[0] = (float)(a / n);
  }
}

// dZ = dH [Z > 0]
__global__ void k_relu_bwd(int64_t m, const float* __restrict__ dH, const float* __restrict__ Z,
                           float* __restrict__ dZ) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    dZ[i] = Z[i] > 0.0f ? dH[i] : 0.0f;
}

// dH_r = dH_{r+1} + dHA[:, :32] (+ dPQ contribution added by a dense layer)
__global__ void k_add_first32(int n, const float* __restrict__ a, const float* __restrict__ hb64,
                              float* __restrict__ out) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < (int64_t)n * 32;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = k >> 5, c = k & 31;
    out[k] = a[k] + hb64[i * 64 + c];
  }
}
__global__ void k_take_last32(int n, const float* __restrict__ hb64, float* __restrict__ out) {
  for (int64_t k = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; k < (int64_t)n * 32;
       k += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = k >> 5, c = k & 31;
    out[k] = hb64[i * 64 + 32 + c];
  }
}
__global__ void k_add_inplace(int64_t m, const float* __restrict__ a, float* __restrict__ out) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x)
    out[i] += a[i];
}

// ---------------------------------------------------------------- parameters
// BF16 copies of the weight matrices (and transposes) from the FP32 vector.
__global__ void k_pack_weights(const float* __restrict__ th, __bf16* __restrict__ wb) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  // W_e padded to [32][32]
  if (t < 32 * 32) {
    const int n = t / 32, k = t % 32;
    wb[net::kWeB + t] = (__bf16)(k < 5 ? th[net::kWe + n * 5 + k] : 0.0f);
  }
  for (int r = 0; r < net::kRounds; ++r) {
    const int ro = net::round_ofs(r), bo = net::round_bofs(r);
    if (t < 64 * 32) {  // AB [64][32] and its transpose [32][64]
      const int n = t / 32, k = t % 32;
      const float v = n < 32 ? th[ro + net::kA + n * 32 + k] : th[ro + net::kBm + (n - 32) * 32 + k];
      wb[bo + net::kABb + t] = (__bf16)v;
      wb[bo + net::kABTb + k * 64 + n] = (__bf16)v;
    }
    if (t < 32 * 64) {  // U [32][64] and its transpose [64][32]
      const int n = t / 64, k = t % 64;
      const float v = th[ro + net::kU + n * 64 + k];
      wb[bo + net::kUb + t] = (__bf16)v;
      wb[bo + net::kUTb + k * 32 + n] = (__bf16)v;
    }
  }
}

__global__ void k_adam(int n, float* __restrict__ th, const float* __restrict__ g,
                       float* __restrict__ m, float* __restrict__ v, float lr, float b1, float b2,
                       float eps, float c1, float c2) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    th[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  }
}

inline int nblocks(int64_t work, int per, int cap = 4096) {
  int64_t g = (work + per - 1) / per;
  return (int)(g < 1 ? 1 : (g > cap ? cap : g));
}

}  // namespace

// ---------------------------------------------------------------- host side

namespace net {

size_t workspace_floats(int n, int nnz) {
  Buffers B;
  return B.carve(nullptr, n, nnz);
}

// Lays the buffers out from base (64-float aligned each) and returns the
// number of floats used; with base == nullptr only the size is computed.
size_t Buffers::carve(float* base, int n, int nnz) {
  const size_t N = n;
  size_t used = 0;
  auto take = [&](size_t k) {
    float* q = base ? base + used : nullptr;
    used += (k + 63) & ~(size_t)63;
    return q;
  };
  Xf = take(32 * N);
  Z0 = take(32 * N);
  for (int r = 0; r <= kRounds; ++r) H[r] = take(32 * N);
  for (int r = 0; r < kRounds; ++r) PQ[r] = take(64 * N);
  for (int r = 0; r < kRounds; ++r) A[r] = take(32 * N);
  for (int r = 0; r < kRounds; ++r) Z[r] = take(32 * N);
  dy = take(N);
  dH = take(32 * N);
  dHb = take(32 * N);
  dZ = take(32 * N);
  dHA = take(64 * N);
  dPQ = take(64 * N);
  ef = reinterpret_cast<float4*>(take(4 * (size_t)nnz));
  deg_inv = take(N);
  grad = take(kParams);
  wpart = take((size_t)nblocks(n, kRowsPerBlock) * (64 * 64 + 64));
  epart = take((size_t)nblocks(n, kB / 32) * 128);
  q = reinterpret_cast<double*>(take(2 * N));
  return used;
}

void launch_extrapolate(int n, const double* h0, const double* h1, const double* h2,
                        const uint8_t* nat, double* q, hipStream_t s) {
  k_extrapolate<<<nblocks(n, kB, 1024), kB, 0, s>>>(n, h0, h1, h2, nat, q);
}

void launch_edge_features(const DLevel& C, double hbar, const Buffers& B, hipStream_t s) {
  k_edge_features<<<nblocks(C.n, kB), kB, 0, s>>>(C, (float)(1.0 / hbar), B.ef, B.deg_inv);
}

void launch_pack(const float* theta, __bf16* wb, hipStream_t s) {
  k_pack_weights<<<8, kB, 0, s>>>(theta, wb);
}

void launch_forward(const DLevel& C, const double* Kval, const float* th, const __bf16* wb,
                    const Buffers& B, const double* b, const double* const hist[4], double hbar,
                    double* dpart, double* scal, hipStream_t s) {
  const int n = C.n;
  const int nb = nblocks(n, kB, 1024);
  k_net_stats<<<nb, kB, 0, s>>>(n, b, hist[0], hist[1], hist[2], hist[3], dpart);
  k_net_features<<<nb, kB, 0, s>>>(C, Kval, dpart, nb, hbar, b, hist[0], hist[1], hist[2],
                                   hist[3], B.Xf, B.q, scal);
  const int gd = nblocks(n, 64);
  k_dense<32, 0, 32, 1><<<gd, kB, 0, s>>>(n, B.Xf, nullptr, wb + kWeB, th + kCe, nullptr, B.Z0,
                                          B.H[0]);
  const int ge = nblocks(n, kB / 32);
  for (int r = 0; r < kRounds; ++r) {
    const float* P = th + round_ofs(r);
    const __bf16* W = wb + round_bofs(r);
    k_dense<32, 0, 64, 0><<<gd, kB, 0, s>>>(n, B.H[r], nullptr, W + kABb, nullptr, nullptr,
                                            nullptr, B.PQ[r]);
    k_edge_fwd<<<ge, kB, 0, s>>>(C, B.ef, B.deg_inv, B.PQ[r], P + kC, P + kD, B.A[r]);
    k_dense<32, 32, 32, 2><<<gd, kB, 0, s>>>(n, B.H[r], B.A[r], W + kUb, P + kV, B.H[r], B.Z[r],
                                             B.H[r + 1]);
  }
}

void launch_decode(const DLevel& C, const float* th, const Buffers& B, const double* scal,
                   const double* target, double* guess, const uint8_t* nat, double* lpart,
                   hipStream_t s) {
  const int nb = nblocks(C.n, kB, 1024);
  if (target) k_target_sq<<<nb, kB, 0, s>>>(C.n, B.q, scal, target, lpart + nb);
  k_decoder<<<nb, kB, 0, s>>>(C.n, B.H[kRounds], th + kW, th + kCd, scal, B.q, target,
                              lpart + nb, nb, B.dy, guess, nat, lpart);
}

void launch_backward(const DLevel& C, const float* th, const __bf16* wb, const Buffers& B,
                     const double* lpart, float* loss, hipStream_t s) {
  const int n = C.n;
  const int nb = nblocks(n, kB, 1024);
  const int ge = nblocks(n, kB / 32);
  const int gd = nblocks(n, 64);
  const int gw = nblocks(n, kRowsPerBlock);
  const int gv = nblocks((int64_t)n * 32, kB);
  float* grad = B.grad;
  k_decoder_bwd<<<ge, kB, 0, s>>>(n, B.H[kRounds], th + kW, B.dy, B.dH, B.epart);
  k_decoder_grad_reduce<<<1, 128, 0, s>>>(B.epart, ge, grad, kW, kCd, lpart, nb, n, loss);
  // dH holds the gradient with respect to H[r + 1]
  for (int r = kRounds - 1; r >= 0; --r) {
    const int ro = round_ofs(r);
    const __bf16* W = wb + round_bofs(r);
    const float* P = th + ro;
    k_relu_bwd<<<gv, kB, 0, s>>>((int64_t)n * 32, B.dH, B.Z[r], B.dZ);
    k_wgrad<32, 32, 32><<<gw, kB, 0, s>>>(n, kRowsPerBlock, B.dZ, B.H[r], B.A[r], B.wpart);
    k_wgrad_reduce<<<8, kB, 0, s>>>(B.wpart, gw, 32, 64, 64, grad, ro + kU, ro + kV);
    // [dh | da] = dZ U
    k_dense<32, 0, 64, 0><<<gd, kB, 0, s>>>(n, B.dZ, nullptr, W + kUTb, nullptr, nullptr, nullptr,
                                            B.dHA);
    k_add_first32<<<gv, kB, 0, s>>>(n, B.dH, B.dHA, B.dHb);  // dHb = dH + dh
    k_take_last32<<<gv, kB, 0, s>>>(n, B.dHA, B.dZ);         // dZ <- da
    k_edge_bwd<<<ge, kB, 0, s>>>(C, B.ef, B.deg_inv, B.PQ[r], P + kC, P + kD, B.dZ, B.dPQ,
                                 B.epart);
    k_edge_grad_reduce<<<1, 128, 0, s>>>(B.epart, ge, grad, ro + kC, ro + kD);
    k_wgrad<32, 0, 64><<<gw, kB, 0, s>>>(n, kRowsPerBlock, B.dPQ, B.H[r], nullptr, B.wpart);
    k_wgrad_reduce<<<8, kB, 0, s>>>(B.wpart, gw, 64, 32, 32, grad, ro + kA, -1);
    // dH_r = dHb + dPQ [A; B]
    k_dense<64, 0, 32, 0><<<gd, kB, 0, s>>>(n, B.dPQ, nullptr, W + kABTb, nullptr, nullptr,
                                            nullptr, B.dH);
    k_add_inplace<<<gv, kB, 0, s>>>((int64_t)n * 32, B.dHb, B.dH);
  }
  // encoder
  k_relu_bwd<<<gv, kB, 0, s>>>((int64_t)n * 32, B.dH, B.Z0, B.dZ);
  k_wgrad<32, 0, 32><<<gw, kB, 0, s>>>(n, kRowsPerBlock, B.dZ, B.Xf, nullptr, B.wpart);
  k_wgrad_reduce<<<8, kB, 0, s>>>(B.wpart, gw, 32, 32, 5, grad, kWe, kCe);
}

void launch_adam(float* th, const float* g, float* m, float* v, int step, float lr,
                 hipStream_t s) {
  const float b1 = 0.9f, b2 = 0.999f;
  const float c1 = 1.0f - std::pow(b1, (float)step), c2 = 1.0f - std::pow(b2, (float)step);
  k_adam<<<nblocks(kParams, kB), kB, 0, s>>>(kParams, th, g, m, v, lr, b1, b2, 1e-8f, c1, c2);
}

}  // namespace net
}  // namespace cgp
