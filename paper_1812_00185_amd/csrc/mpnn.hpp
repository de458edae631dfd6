// Internal declarations of the learned-initial-guess network (mpnn.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "device.hpp"

namespace cgp {
namespace net {

constexpr int kHidden = 32;
constexpr int kRounds = 3;
constexpr int kFeat = 5;
constexpr int kRowsPerBlock = 256;  // rows per block in the weight-gradient products

// flat FP32 parameter vector: W_e [32][5], c_e [32], per round
// A [32][32], B [32][32], C [32][3], d [32], U [32][64], v [32]; w [32], c
constexpr int kWe = 0;
constexpr int kCe = kWe + 32 * 5;
constexpr int kRound0 = kCe + 32;
constexpr int kA = 0;
constexpr int kBm = kA + 32 * 32;
constexpr int kC = kBm + 32 * 32;
constexpr int kD = kC + 32 * 3;
constexpr int kU = kD + 32;
constexpr int kV = kU + 32 * 64;
constexpr int kRoundSize = kV + 32;
constexpr int kW = kRound0 + kRounds * kRoundSize;
constexpr int kCd = kW + 32;
constexpr int kParams = kCd + 1;
static_assert(kParams == 12993, "parameter count");
constexpr __host__ __device__ int round_ofs(int r) { return kRound0 + r * kRoundSize; }

// BF16 weight copies: W_e padded [32][32]; per round AB [64][32], AB^T
// [32][64], U [32][64], U^T [64][32]
constexpr int kWeB = 0;
constexpr int kABb = 0;
constexpr int kABTb = kABb + 64 * 32;
constexpr int kUb = kABTb + 32 * 64;
constexpr int kUTb = kUb + 32 * 64;
constexpr int kRoundBSize = kUTb + 64 * 32;
constexpr int kWeightsB = 32 * 32 + kRounds * kRoundBSize;
constexpr __host__ __device__ int round_bofs(int r) { return 32 * 32 + r * kRoundBSize; }

// FP32 activations and gradients of one coarse graph (carved from the
// workspace).
struct Buffers {
  float *Xf = nullptr, *Z0 = nullptr;
  float* H[kRounds + 1] = {};
  float* PQ[kRounds] = {};
  float* A[kRounds] = {};
  float* Z[kRounds] = {};
  float *dy = nullptr, *dH = nullptr, *dHb = nullptr, *dZ = nullptr, *dHA = nullptr,
        *dPQ = nullptr;
  float4* ef = nullptr;
  float* deg_inv = nullptr;
  float* grad = nullptr;
  float *wpart = nullptr, *epart = nullptr;
  double* q = nullptr;  // quadratic extrapolation of the history [n]
  size_t carve(float* base, int n, int nnz);
};

size_t workspace_floats(int n, int nnz);

void launch_edge_features(const DLevel& C, double hbar, const Buffers& B, hipStream_t s);
// q = 3 h0 - 3 h1 + h2 (0 where nat[i], nat may be null)
void launch_extrapolate(int n, const double* h0, const double* h1, const double* h2,
                        const uint8_t* nat, double* q, hipStream_t s);
void launch_pack(const float* theta, __bf16* wb, hipStream_t s);
// scales, the extrapolation B.q, inputs, encoder and the three rounds; Kval:
// the solver's coarse operator (residual feature); dpart: >= 5 * 1024
// doubles of reduction scratch; scal[0..3] receives (s_b, s, s_1, s_2)
void launch_forward(const DLevel& C, const double* Kval, const float* theta, const __bf16* wb,
                    const Buffers& B, const double* b, const double* const hist[4], double hbar,
                    double* dpart, double* scal, hipStream_t s);
// decoder: with a target the loss partials and dy, else the guess; lpart:
// >= 2 * 1024 doubles
void launch_decode(const DLevel& C, const float* theta, const Buffers& B, const double* scal,
                   const double* target, double* guess, const uint8_t* nat, double* lpart,
                   hipStream_t s);
void launch_backward(const DLevel& C, const float* theta, const __bf16* wb, const Buffers& B,
                     const double* lpart, float* loss, hipStream_t s);
void launch_adam(float* theta, const float* grad, float* m, float* v, int step, float lr,
                 hipStream_t s);

}  // namespace net

// FP64 residuals of two candidate initial guesses against the coarse system;
// the smaller one (the first on ties) is copied into out and *chose set to 0
// (first) or 1 (second).
void launch_guard(const DLevel& C, const double* Kval, const double* b, const double* cand,
                  const double* prev, double* out, int32_t* chose, double* part, int nb,
                  hipStream_t s);

}  // namespace cgp
