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
// LDS row strides of the bf16 tiles, padded by 8 elements (16 bytes) so that
// the 16 rows an operand fragment reads start in different bank groups
constexpr int kXS = kInP + 8, kHS = kH + 8, kOS = kOutP + 8;
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

// Weights in LDS, bf16, transposed ([n][k]) so that the B operand of a tile
// (four consecutive k of one column n) is one 8-byte read, like the A operand.
struct alignas(16) Weights {
  alignas(16) unsigned short w1t[kH][kXS];    // W1^T, k padded 18 -> 32 with zeros
  alignas(16) unsigned short w2t[kH][kHS];    // W2^T
  alignas(16) unsigned short w3t[kOutP][kHS]; // W3^T, n padded 2 -> 16 with zeros
  float b1[kH], b2[kH], b3[kOutP];
};

// Per-wave activations of one 16-sample tile.
struct Act {
  alignas(16) unsigned short h1[16][kHS];
  alignas(16) unsigned short h2[16][kHS];
};

__device__ inline void stage_weights(Weights &W, const float *p) {
  for (int i = threadIdx.x; i < kH * kXS; i += blockDim.x) {
    const int n = i / kXS, k = i % kXS;
    W.w1t[n][k] = k < kIn ? f2bf(p[kOffW1 + k * kH + n]) : 0;
  }
  for (int i = threadIdx.x; i < kH * kHS; i += blockDim.x) {
    const int n = i / kHS, k = i % kHS;
    W.w2t[n][k] = k < kH ? f2bf(p[kOffW2 + k * kH + n]) : 0;
  }
  for (int i = threadIdx.x; i < kOutP * kHS; i += blockDim.x) {
    const int n = i / kHS, k = i % kHS;
    W.w3t[n][k] = (n < kOut && k < kH) ? f2bf(p[kOffW3 + k * kOut + n]) : 0;
  }
  for (int i = threadIdx.x; i < kH; i += blockDim.x) {
    W.b1[i] = p[kOffB1 + i];
    W.b2[i] = p[kOffB2 + i];
  }
  for (int i = threadIdx.x; i < kOutP; i += blockDim.x) W.b3[i] = i < kOut ? p[kOffB3 + i] : 0.0f;
}

// Copy of a packed Weights image (made once by k_mlp_pack) into LDS with
// coalesced 16-byte loads.
__device__ inline void load_packed(Weights &W, const Weights *g) {
  static_assert(sizeof(Weights) % 16 == 0, "whole 16-byte words");
  const int4 *src = reinterpret_cast<const int4 *>(g);
  int4 *dst = reinterpret_cast<int4 *>(&W);
  for (int i = threadIdx.x; i < (int)(sizeof(Weights) / 16); i += blockDim.x) dst[i] = src[i];
}

// One 16x16 output tile D = A (16 x K) * B (K x 16) with A row-major [16][lda]
// and B given transposed, Bt row-major [n][ldb] (rows n0 .. n0 + 15), both
// bf16 in LDS; K a multiple of 16, lda and ldb multiples of 4.
__device__ inline f32x4 tile_gemm(const unsigned short *A, int lda, const unsigned short *Bt, int ldb, int n0, int K) {
  const int lane = threadIdx.x & 63;
  const int r = lane & 15, g = lane >> 4;
  f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
  for (int k0 = 0; k0 < K; k0 += 16) {
    const bf16x4 a = *reinterpret_cast<const bf16x4 *>(A + r * lda + k0 + 4 * g);
    const bf16x4 b = *reinterpret_cast<const bf16x4 *>(Bt + (n0 + r) * ldb + k0 + 4 * g);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
  }
  return acc;
}

// Makes this wavefront's LDS writes visible to its own later reads (no
// workgroup barrier): for tiles that only one wavefront touches.
__device__ inline void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

// Forward of the 16 samples in x (bf16, row stride kXS, columns kIn .. kInP - 1 zero).
// Fills A.h1, A.h2 (post-ReLU) and returns the raw outputs of rows
// 4 (lane / 16) + j, column lane % 16 (columns 0 and 1 are the outputs).
// kWaveOnly: x and A belong to this wavefront alone, so wavefront-level
// ordering suffices; otherwise every wavefront of the workgroup must call it
// the same number of times (workgroup barriers).
template <bool kWaveOnly = false>
__device__ inline f32x4 forward16(const Weights &W, const unsigned short *x, Act &A) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, g = lane >> 4;
#pragma unroll
  for (int nt = 0; nt < kH / 16; ++nt) {
    const f32x4 acc = tile_gemm(x, kXS, &W.w1t[0][0], kXS, 16 * nt, kInP);
#pragma unroll
    for (int j = 0; j < 4; ++j) A.h1[4 * g + j][16 * nt + col] = f2bf(fmaxf(acc[j] + W.b1[16 * nt + col], 0.0f));
  }
  if (kWaveOnly) wave_lds_sync();
  else __syncthreads();
#pragma unroll
  for (int nt = 0; nt < kH / 16; ++nt) {
    const f32x4 acc = tile_gemm(&A.h1[0][0], kHS, &W.w2t[0][0], kHS, 16 * nt, kH);
#pragma unroll
    for (int j = 0; j < 4; ++j) A.h2[4 * g + j][16 * nt + col] = f2bf(fmaxf(acc[j] + W.b2[16 * nt + col], 0.0f));
  }
  if (kWaveOnly) wave_lds_sync();
  else __syncthreads();
  f32x4 acc = tile_gemm(&A.h2[0][0], kHS, &W.w3t[0][0], kHS, 0, kH);
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] += W.b3[col];
  return acc;
}

// The same forward for inference, with every layer computed transposed
// (H^T = W^T X^T: the weights are the A operand, the samples the columns):
// then the output tile of one layer is, lane for lane, the B operand of the
// next, and the activations stay in registers.  x holds the 16 samples as
// rows (bf16, row stride kXS, columns kIn .. kInP - 1 zero).  Lane l
// receives the outputs 4 (l / 16) + j of sample l % 16, so lanes 0..15 hold
// the two outputs in elements 0 and 1.
__device__ inline f32x4 forward_t16(const Weights &W, const unsigned short *x) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, g = lane >> 4;
  bf16x4 h1[kH / 16], h2[kH / 16];
#pragma unroll
  for (int nt = 0; nt < kH / 16; ++nt) {
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int k0 = 0; k0 < kInP; k0 += 16) {
      const bf16x4 a = *reinterpret_cast<const bf16x4 *>(&W.w1t[16 * nt + col][k0 + 4 * g]);
      const bf16x4 b = *reinterpret_cast<const bf16x4 *>(x + col * kXS + k0 + 4 * g);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) h1[nt][j] = (short)f2bf(fmaxf(acc[j] + W.b1[16 * nt + 4 * g + j], 0.0f));
  }
#pragma unroll
  for (int nt = 0; nt < kH / 16; ++nt) {
    f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int kt = 0; kt < kH / 16; ++kt) {
      const bf16x4 a = *reinterpret_cast<const bf16x4 *>(&W.w2t[16 * nt + col][16 * kt + 4 * g]);
      acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, h1[kt], acc, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) h2[nt][j] = (short)f2bf(fmaxf(acc[j] + W.b2[16 * nt + 4 * g + j], 0.0f));
  }
  f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int kt = 0; kt < kH / 16; ++kt) {
    const bf16x4 a = *reinterpret_cast<const bf16x4 *>(&W.w3t[col][16 * kt + 4 * g]);
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, h2[kt], acc, 0, 0, 0);
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) acc[j] += W.b3[4 * g + j];
  return acc;
}

__device__ inline float head_mu(float o0) { return 1.0f / (1.0f + __expf(-o0)); }
__device__ inline float head_sd(float o1) { return (o1 > 20.0f ? o1 : log1pf(__expf(o1))) + kSdFloor; }

}  // namespace mlp
}  // namespace stiv
