// Inference and training kernels of the learned contact-time bracket
// (perceptron 18 -> 64 -> 64 -> 2, bf16 matrix-core tiles from mlp_tile.h):
// batched forward, gradient of the mean Gaussian negative log-likelihood
// with a deterministic cross-workgroup reduction, and Adam on FP32 master
// weights.
#include "mlp_tile.h"
#include "stiv_common.h"

namespace stiv {

namespace {

using namespace mlp;

constexpr int kWaves = 4, kThreads = 64 * kWaves;

struct WaveBuf {
  alignas(16) unsigned short x[16][kXS];  // [sample][k]
  Act a;
  float o[16][kOut];
};

__device__ inline void load_x(WaveBuf &B, const float *x, int64_t s0, int64_t n) {
  const int lane = threadIdx.x & 63;
  for (int i = lane; i < 16 * kInP; i += 64) {
    const int r = i / kInP, k = i % kInP;
    const int64_t s = s0 + r;
    B.x[r][k] = (k < kIn && s < n) ? f2bf(x[s * kIn + k]) : 0;
  }
}

__device__ inline void forward_tile(const Weights &W, WaveBuf &B) {
  const int lane = threadIdx.x & 63;
  const int col = lane & 15, g = lane >> 4;
  const f32x4 o = forward16(W, &B.x[0][0], B.a);
  if (col < kOut)
#pragma unroll
    for (int j = 0; j < 4; ++j) B.o[4 * g + j][col] = o[j];
  __syncthreads();
}

__global__ __launch_bounds__(kThreads) void k_mlp_forward(const float *params, const float *x, int64_t n,
                                                          float *out) {
  __shared__ Weights W;
  __shared__ WaveBuf buf[kWaves];
  stage_weights(W, params);
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  WaveBuf &B = buf[wave];
  const int64_t tiles = (n + 15) / 16;
  // the tile loop has the same trip count for every wave of the workgroup
  for (int64_t t0 = (int64_t)blockIdx.x * kWaves; t0 < tiles; t0 += (int64_t)gridDim.x * kWaves) {
    const int64_t t = t0 + wave;
    load_x(B, x, 16 * t, t < tiles ? n : 0);
    __syncthreads();
    // the inference form of the forward (activations in registers), the
    // one the narrow phase runs
    const f32x4 o = forward_t16(W, &B.x[0][0]);
    if (t < tiles && lane < 16) {
      const int64_t s = 16 * t + lane;
      if (s < n) {
        out[s * kOut] = o[0];
        out[s * kOut + 1] = o[1];
      }
    }
    __syncthreads();
  }
}

// Loss and output gradient of one sample (target s in [0,1]).
__device__ inline float head_grad(float o0, float o1, float s, float *d0, float *d1) {
  const float mu = head_mu(o0);
  const float sd = head_sd(o1);
  const float z = (s - mu) / sd;
  *d0 = -z / sd * mu * (1.0f - mu);
  *d1 = (1.0f / sd - z * z / sd) * (1.0f / (1.0f + __expf(-o1)));
  return 0.5f * z * z + logf(sd);
}

// Gradient of the mean loss over n samples.  Each workgroup writes its
// partial sums to part[blockIdx.x][kNParam + 1] (last entry: loss sum); a
// second kernel adds the partials in workgroup order.  Sums inside a
// workgroup go wave by wave in a fixed order, so the result is reproducible.
__global__ __launch_bounds__(kThreads) void k_mlp_grad(const float *params, const float *x, const float *target,
                                                       int64_t n, float *part) {
  __shared__ Weights W;
  __shared__ WaveBuf buf[kWaves];
  __shared__ alignas(16) unsigned short dO[kWaves][16][kOS];  // output gradient (bf16), columns 0..1
  __shared__ alignas(16) unsigned short d2[kWaves][16][kHS];  // gradient at the layer-2 pre-activation
  __shared__ alignas(16) unsigned short d1[kWaves][16][kHS];  // gradient at the layer-1 pre-activation
  // W2 and W3 untransposed ([in][out]): the B^T operands of the backward products
  __shared__ alignas(16) unsigned short w2o[kH][kHS];
  __shared__ alignas(16) unsigned short w3o[kH][kOS];
  __shared__ float gsum[kNParam + 1];
  __shared__ float bsum[kWaves][2 * kH + kOut];     // per-wave bias gradients
  stage_weights(W, params);
  for (int i = threadIdx.x; i < kNParam + 1; i += blockDim.x) gsum[i] = 0.0f;
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int col = lane & 15, g = lane >> 4;
  WaveBuf &B = buf[wave];
  for (int i = threadIdx.x; i < kH * kH; i += blockDim.x) w2o[i / kH][i % kH] = W.w2t[i % kH][i / kH];
  for (int i = threadIdx.x; i < kH * kOutP; i += blockDim.x) w3o[i / kOutP][i % kOutP] = W.w3t[i % kOutP][i / kOutP];
  for (int i = lane; i < 2 * kH + kOut; i += 64) bsum[wave][i] = 0.0f;
  __syncthreads();
  // per-lane accumulators of the dW tiles: dW2 (4 x 4 tiles), dW1 (2 x 4), dW3 (4 x 1)
  f32x4 aw2[16], aw1[8], aw3[4];
  for (int i = 0; i < 16; ++i) aw2[i] = f32x4{0, 0, 0, 0};
  for (int i = 0; i < 8; ++i) aw1[i] = f32x4{0, 0, 0, 0};
  for (int i = 0; i < 4; ++i) aw3[i] = f32x4{0, 0, 0, 0};
  float lsum = 0.0f;
  const int64_t tiles = (n + 15) / 16;
  for (int64_t t0 = (int64_t)blockIdx.x * kWaves; t0 < tiles; t0 += (int64_t)gridDim.x * kWaves) {
    const int64_t t = t0 + wave;
    load_x(B, x, 16 * t, t < tiles ? n : 0);
    for (int i = lane; i < 16 * kOutP; i += 64) dO[wave][i / kOutP][i % kOutP] = 0;
    __syncthreads();
    forward_tile(W, B);
    // output gradient of the mean (scaled by 1/n)
    if (lane < 16) {
      const int64_t s = 16 * t + lane;
      if (t < tiles && s < n) {
        float g0, g1;
        lsum += head_grad(B.o[lane][0], B.o[lane][1], target[s], &g0, &g1);
        dO[wave][lane][0] = f2bf(g0 / (float)n);
        dO[wave][lane][1] = f2bf(g1 / (float)n);
      }
    }
    __syncthreads();
    // d2 = (dO W3^T) * relu'(h2)
    for (int nt = 0; nt < kH / 16; ++nt) {
      const f32x4 acc = tile_gemm(&dO[wave][0][0], kOS, &w3o[0][0], kOS, 16 * nt, kOutP);
      for (int j = 0; j < 4; ++j) {
        const int r = 4 * g + j, c = 16 * nt + col;
        d2[wave][r][c] = B.a.h2[r][c] ? f2bf(acc[j]) : 0;
      }
    }
    __syncthreads();
    // d1 = (d2 W2^T) * relu'(h1)
    for (int nt = 0; nt < kH / 16; ++nt) {
      const f32x4 acc = tile_gemm(&d2[wave][0][0], kHS, &w2o[0][0], kHS, 16 * nt, kH);
      for (int j = 0; j < 4; ++j) {
        const int r = 4 * g + j, c = 16 * nt + col;
        d1[wave][r][c] = B.a.h1[r][c] ? f2bf(acc[j]) : 0;
      }
    }
    __syncthreads();
    // weight gradients dW = act^T delta, contracted over the 16 samples:
    // A[i][k] = act[k][i0 + i], B[k][n] = delta[k][n0 + n]
    for (int it = 0; it < 4; ++it)
      for (int nt = 0; nt < 4; ++nt) {
        bf16x4 a, b;
        for (int j = 0; j < 4; ++j) {
          a[j] = (short)B.a.h1[4 * g + j][16 * it + col];
          b[j] = (short)d2[wave][4 * g + j][16 * nt + col];
        }
        aw2[it * 4 + nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, aw2[it * 4 + nt], 0, 0, 0);
      }
    for (int it = 0; it < 2; ++it)
      for (int nt = 0; nt < 4; ++nt) {
        bf16x4 a, b;
        for (int j = 0; j < 4; ++j) {
          a[j] = (short)B.x[4 * g + j][16 * it + col];
          b[j] = (short)d1[wave][4 * g + j][16 * nt + col];
        }
        aw1[it * 4 + nt] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, aw1[it * 4 + nt], 0, 0, 0);
      }
    for (int it = 0; it < 4; ++it) {
      bf16x4 a, b;
      for (int j = 0; j < 4; ++j) {
        a[j] = (short)B.a.h2[4 * g + j][16 * it + col];
        b[j] = (short)dO[wave][4 * g + j][col];
      }
      aw3[it] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, aw3[it], 0, 0, 0);
    }
    // bias gradients: column sums of the deltas (each lane owns its columns)
    {
      float s1 = 0.0f, s2 = 0.0f;
      for (int k = 0; k < 16; ++k) {
        s1 += bf2f(d1[wave][k][lane]);
        s2 += bf2f(d2[wave][k][lane]);
      }
      bsum[wave][lane] += s1;
      bsum[wave][kH + lane] += s2;
      if (lane < kOut) {
        float s3 = 0.0f;
        for (int k = 0; k < 16; ++k) s3 += bf2f(dO[wave][k][lane]);
        bsum[wave][2 * kH + lane] += s3;
      }
    }
    __syncthreads();
  }
  // dW tiles: each lane holds D[4g + j][col] of every tile; waves add in order
  for (int w = 0; w < kWaves; ++w) {
    if (wave == w) {
      for (int it = 0; it < 4; ++it)
        for (int nt = 0; nt < 4; ++nt)
          for (int j = 0; j < 4; ++j)
            gsum[kOffW2 + (16 * it + 4 * g + j) * kH + 16 * nt + col] += aw2[it * 4 + nt][j];
      for (int it = 0; it < 2; ++it)
        for (int nt = 0; nt < 4; ++nt)
          for (int j = 0; j < 4; ++j) {
            const int k = 16 * it + 4 * g + j;
            if (k < kIn) gsum[kOffW1 + k * kH + 16 * nt + col] += aw1[it * 4 + nt][j];
          }
      for (int it = 0; it < 4; ++it)
        for (int j = 0; j < 4; ++j)
          if (col < kOut) gsum[kOffW3 + (16 * it + 4 * g + j) * kOut + col] += aw3[it][j];
      gsum[kOffB1 + lane] += bsum[w][lane];
      gsum[kOffB2 + lane] += bsum[w][kH + lane];
      if (lane < kOut) gsum[kOffB3 + lane] += bsum[w][2 * kH + lane];
      float ls = lsum;
      for (int off = 32; off > 0; off >>= 1) ls += __shfl_xor(ls, off, 64);
      if (lane == 0) gsum[kNParam] += ls;
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < kNParam + 1; i += blockDim.x) part[(int64_t)blockIdx.x * (kNParam + 1) + i] = gsum[i];
}

// The LDS image of the weights (bf16, transposed, padded), made once per model.
__global__ void k_mlp_pack(const float *params, Weights *out) {
  __shared__ Weights W;
  stage_weights(W, params);
  __syncthreads();
  const int4 *src = reinterpret_cast<const int4 *>(&W);
  int4 *dst = reinterpret_cast<int4 *>(out);
  for (int i = threadIdx.x; i < (int)(sizeof(Weights) / 16); i += blockDim.x) dst[i] = src[i];
}

__global__ void k_mlp_reduce(const float *part, int nblocks, float *grad, float *loss, int64_t n) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kNParam + 1; i += gridDim.x * blockDim.x) {
    float s = 0.0f;
    for (int b = 0; b < nblocks; ++b) s += part[(int64_t)b * (kNParam + 1) + i];
    if (i < kNParam) grad[i] = s;
    else if (loss) *loss = s / (float)(n > 0 ? n : 1);
  }
}

__global__ void k_adam(float *p, const float *g, float *m, float *v, int64_t step, float lr, float b1, float b2,
                       float eps) {
  const float c1 = 1.0f - powf(b1, (float)step), c2 = 1.0f - powf(b2, (float)step);
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < kNParam; i += gridDim.x * blockDim.x) {
    m[i] = b1 * m[i] + (1.0f - b1) * g[i];
    v[i] = b2 * v[i] + (1.0f - b2) * g[i] * g[i];
    p[i] -= lr * (m[i] / c1) / (sqrtf(v[i] / c2) + eps);
  }
}

}  // namespace

int mlp_nparam() { return kNParam; }

size_t mlp_packed_bytes() { return sizeof(Weights); }

void launch_mlp_pack(const float *params, void *packed, hipStream_t st) {
  k_mlp_pack<<<1, 256, 0, st>>>(params, reinterpret_cast<Weights *>(packed));
}

void launch_mlp_forward(const float *params, const float *x, int64_t n, float *out, hipStream_t st) {
  int64_t tiles = (n + 15) / 16;
  int64_t g = (tiles + kWaves - 1) / kWaves;
  g = g > 2048 ? 2048 : (g < 1 ? 1 : g);
  k_mlp_forward<<<(int)g, kThreads, 0, st>>>(params, x, n, out);
}

int mlp_grad_blocks(int64_t n) {
  int64_t tiles = (n + 15) / 16;
  int64_t g = (tiles + kWaves - 1) / kWaves;
  return (int)(g > 512 ? 512 : (g < 1 ? 1 : g));
}

void launch_mlp_grad(const float *params, const float *x, const float *target, int64_t n, float *part, float *grad,
                     float *loss, hipStream_t st) {
  const int g = mlp_grad_blocks(n);
  k_mlp_grad<<<g, kThreads, 0, st>>>(params, x, target, n, part);
  k_mlp_reduce<<<(kNParam + 1 + 255) / 256, 256, 0, st>>>(part, g, grad, loss, n);
}

void launch_adam(float *p, const float *g, float *m, float *v, int64_t step, float lr, float b1, float b2, float eps,
                 hipStream_t st) {
  k_adam<<<(kNParam + 255) / 256, 256, 0, st>>>(p, g, m, v, step, lr, b1, b2, eps);
}

}  // namespace stiv
