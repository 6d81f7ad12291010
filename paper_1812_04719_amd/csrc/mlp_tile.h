// Building blocks of the learned contact-time bracket: a 3-layer perceptron
// 18 -> 64 -> 64 -> 2 with bf16 weights and activations and FP32
// accumulation on the matrix cores (v_mfma_f32_16x16x16_bf16).
//
// Parameters (FP32, flat): W1[18][64] b1[64] W2[64][64] b2[64] W3[64][2] b3[2].
// A workgroup converts the weights to bf16 once and keeps them in LDS with
// the padding the 16x16x16 tiles need (K of layer 1 padded 18 -> 32, N of
// layer 3 padded 2 -> 16).  Each wavefront pushes 16 samples at a time
// through the three layers.
//
// Matrix-core operand layout (16x16x16, 64 lanes): lane l supplies
// A[l % 16][4 (l / 16) + j] and B[4 (l / 16) + j][l % 16], j = 0..3, and
// receives D[4 (l / 16) + j][l % 16].
//
// Output head: mu = sigmoid(o0) is the predicted contact time in [0,1] and
// sd = softplus(o1) + 1e-3 its spread; training minimises the Gaussian
// negative log-likelihood 0.5 ((s - mu) / sd)^2 + log sd.
#pragma once
#include <hip/hip_runtime.h>

namespace stiv {
namespace mlp {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kIn = 18, kInP = 32, kH = 64, kOut = 2, kOutP = 16;
constexpr int kOffW1 = 0, kOffB1 = kOffW1 + kIn * kH, kOffW2 = kOffB1 + kH, kOffB2 = kOffW2 + kH * kH,
              kOffW3 = kOffB2 + kH, kOffB3 = kOffW3 + kH * kOut, kNParam = kOffB3 + kOut;
constexpr float kSdFloor = 1e-3f;

__device__ inline unsigned short f2bf(float f) {  // round to nearest even
  unsigned int u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (unsigned short)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}
__device__ inline float bf2f(unsigned short h) { return __uint_as_float((unsigned int)h << 16); }

struct Weights {
  unsigned short w1[kInP][kH];  // [k][n]
  unsigned short w2[kH][kH];
  unsigned short w3[kH][kOutP];
  float b1[kH], b2[kH], b3[kOutP];
};

// Per-wave activations of one 16-sample tile.
struct Act {
  unsigned short h1[16][kH];
  unsigned short h2[16][kH];
};

__device__ inline void stage_weights(Weights &W, const float *p) {
  for (int i = threadIdx.x; i < kInP * kH; i += blockDim.x) {
    const int k = i / kH, n = i % kH;
    W.w1[k][n] = k < kIn ? f2bf(p[kOffW1 + k * kH + n]) : 0;
  }
  for (int i = threadIdx.x; i < kH * kH; i += blockDim.x) W.w2[i / kH][i % kH] = f2bf(p[kOffW2 + i]);
  for (int i = threadIdx.x; i < kH * kOutP; i += blockDim.x) {
    const int k = i / kOutP, n = i % kOutP;
    W.w3[k][n] = n < kOut ? f2bf(p[kOffW3 + k * kOut + n]) : 0;
  }
  for (int i = threadIdx.x; i < kH; i += blockDim.x) {
    W.b1[i] = p[kOffB1 + i];
    W.b2[i] = p[kOffB2 + i];
  }
  for (int i = threadIdx.x; i < kOutP; i += blockDim.x) W.b3[i] = i < kOut ? p[kOffB3 + i] : 0.0f;
}

// One 16x16 output tile D = A (16 x K) * B (K x 16); A and B row-major bf16
// in LDS with leading dimensions lda, ldb; columns [n0, n0+16) of B.
__device__ inline f32x4 tile_gemm(const unsigned short *A, int lda, const unsigned short *B, int ldb, int n0, int K) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    bf16x4 a, b;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      a[j] = (short)A[r * lda + k0 + 4 * g + j];
      b[j] = (short)B[(k0 + 4 * g + j) * ldb + n0 + r];
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// Forward of the 16 samples in x (bf16, row stride kInP, columns >= kIn zero).
// Fills A.h1, A.h2 (post-ReLU) and returns the two raw outputs of row
// 4 (lane / 16) + j in out[j][0..1] for the lanes with lane % 16 < 2 (column
// lane % 16).  Contains workgroup barriers: every wave of the workgroup must
// call it the same number of times.
__device__ inline f32x4 forward16(const Weights &W, const unsigned short *x, Act &A) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, g = lane >> 4;
#pragma unroll
  for (int nt = 0; nt < kH / 16; ++nt) {
    const f32x4 acc = tile_gemm(x, kInP, &W.w1[0][0], kH, 16 * nt, kInP);
#pragma unroll
    for (int j = 0; j < 4; ++j) A.h1[4 * g + j][16 * nt + col] = f2bf(fmaxf(acc[j] + W.b1[16 * nt + col], 0.0f));
  }
  __syncthreads();
#pragma unroll
  for (int nt = 0; nt < kH / 16; ++nt) {
    const f32x4 acc = tile_gemm(&A.h1[0][0], kH, &W.w2[0][0], kH, 16 * nt, kH);
#pragma unroll
    for (int j = 0; j < 4; ++j) A.h2[4 * g + j][16 * nt + col] = f2bf(fmaxf(acc[j] + W.b2[16 * nt + col], 0.0f));
  }
  __syncthreads();
  f32x4 acc = tile_gemm(&A.h2[0][0], kH, &W.w3[0][0], kOutP, 0, kH);
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] += W.b3[col];
  return acc;
}

__device__ inline float head_mu(float o0) { return 1.0f / (1.0f + __expf(-o0)); }
__device__ inline float head_sd(float o1) { return (o1 > 20.0f ? o1 : log1pf(__expf(o1))) + kSdFloor; }

}  // namespace mlp
}  // namespace stiv
