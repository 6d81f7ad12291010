// K0: space-time bounding boxes (Sec. 3.3.1; Alg. 2, getBoundingBox).
//
// A vesicle's box is the componentwise min/max over all its vertices at t_n
// and t_{n+1}, inflated by h = d/2 per side.  min/max are exact, so the
// FP64 box is bit-identical to any other correct evaluation.  Patch boxes
// (the same over the vertices referenced by a patch's triangles) feed the
// primitive broad phase.  One workgroup streams one vesicle's SoA positions
// with coalesced 8-byte lanes, once; this is the one stage that reads every
// byte of X0 and X1.
#include "stiv_common.h"

namespace stiv {

namespace {

__device__ inline double wave_min(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ inline double wave_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
  return v;
}

// Order-preserving map of doubles to unsigned 64-bit keys (for exact
// min/max with integer LDS atomics); finite inputs only.
__device__ inline unsigned long long okey(double x) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(x);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__device__ inline double okey_inv(unsigned long long k) {
  const unsigned long long b = (k >> 63) ? (k & 0x7fffffffffffffffull) : ~k;
  return __longlong_as_double((long long)b);
}

// Folds vertex bounds (keys) into a patch's LDS box.  The box only shrinks
// toward its final value, so a vertex that does not beat the value read now
// cannot beat the final one: its atomic is skipped (most vertices of a patch
// are not extreme, and neighbouring lanes often hit the same patch).
__device__ inline void fold_box(unsigned long long (*pk)[6], int q, const unsigned long long kl[3],
                                const unsigned long long ku[3]) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const unsigned long long lo = __hip_atomic_load(&pk[q][c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    const unsigned long long hi = __hip_atomic_load(&pk[q][3 + c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
    if (kl[c] < lo) atomicMin(&pk[q][c], kl[c]);
    if (ku[c] > hi) atomicMax(&pk[q][3 + c], ku[c]);
  }
}

// One workgroup per vesicle: each thread streams vertices (coalesced SoA
// loads of X0 and X1), folds them into the vesicle box and, through the
// vertex -> patch incidence (packed four to a vertex), into the LDS boxes of
// the patches that reference the vertex.
// MAXP bounds the patches of any vesicle's topology (LDS is sized for it, so
// small meshes keep more workgroups resident).
constexpr int kBoxU = 4;

template <int MAXP>
__global__ __launch_bounds__(256) void k_boxes(DevScene S, DevTopo T, double h, const int64_t *ves_patch_off,
                                               double *ves_box, double *patch_box, Counters *cnt) {
  __shared__ unsigned long long pk[MAXP][6];  // lo as key, hi as key
  __shared__ double red[4][6];
  __shared__ int bad_any;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nv_all = S.n_vtx;
  for (int v = blockIdx.x; v < S.n_ves; v += gridDim.x) {
    const int base = S.vtx_off[v];
    const int nvv = S.vtx_off[v + 1] - base;
    const int t = S.topo_id[v];
    const int np = T.patch_off[t + 1] - T.patch_off[t];
    const int vb = T.vbase[t];
    for (int k = threadIdx.x; k < np; k += blockDim.x)
      for (int c = 0; c < 3; ++c) { pk[k][c] = ~0ull; pk[k][3 + c] = 0ull; }
    if (threadIdx.x == 0) bad_any = 0;
    __syncthreads();
    double lo[3], hi[3];
    for (int c = 0; c < 3; ++c) { lo[c] = INFINITY; hi[c] = -INFINITY; }
    int bad = 0;
    // kBoxU vertices per thread at a time: every load of the batch (positions
    // and the packed patch list) is issued before any of them is used, so a
    // workgroup waits for memory once per batch, not twice per vertex
    for (int i0 = threadIdx.x; i0 < nvv; i0 += kBoxU * blockDim.x) {
      double x0[kBoxU][3], x1[kBoxU][3];
      int4 q4[kBoxU];
#pragma unroll
      for (int k = 0; k < kBoxU; ++k) {
        const int i = i0 + k * blockDim.x;
        const bool in = i < nvv;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          x0[k][c] = in ? S.x0[c * nv_all + base + i] : 0.0;
          x1[k][c] = in ? S.x1[c * nv_all + base + i] : 0.0;
        }
        q4[k] = in ? T.vp4[vb + i] : make_int4(-1, -1, -1, -1);
      }
#pragma unroll
      for (int k = 0; k < kBoxU; ++k) {
        const int i = i0 + k * blockDim.x;
        if (i >= nvv) break;
        double l[3], u[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double a = x0[k][c], b = x1[k][c];
          bad |= !(isfinite(a) && isfinite(b));
          l[c] = fmin(a, b);
          u[c] = fmax(a, b);
          lo[c] = fmin(lo[c], l[c]);
          hi[c] = fmax(hi[c], u[c]);
        }
        const unsigned long long kl[3] = {okey(l[0]), okey(l[1]), okey(l[2])};
        const unsigned long long ku[3] = {okey(u[0]), okey(u[1]), okey(u[2])};
        const int qs[4] = {q4[k].x, q4[k].y, q4[k].z, q4[k].w};
        if (qs[3] == -2) {  // more than four patches: the full list
          for (int e = T.vp_off[vb + i]; e < T.vp_off[vb + i + 1]; ++e) fold_box(pk, T.vp[e], kl, ku);
        } else {
#pragma unroll
          for (int j = 0; j < 4; ++j) {
            if (qs[j] < 0) break;
            fold_box(pk, qs[j], kl, ku);
          }
        }
      }
    }
    for (int c = 0; c < 3; ++c) {
      lo[c] = wave_min(lo[c]);
      hi[c] = wave_max(hi[c]);
    }
    if (lane == 0)
      for (int c = 0; c < 3; ++c) { red[wave][c] = lo[c]; red[wave][3 + c] = hi[c]; }
    if (bad) atomicOr(&bad_any, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int c = 0; c < 3; ++c) {
        double l = red[0][c], u = red[0][3 + c];
        for (int w = 1; w < 4; ++w) { l = fmin(l, red[w][c]); u = fmax(u, red[w][3 + c]); }
        ves_box[6 * (int64_t)v + c] = l - h;
        ves_box[6 * (int64_t)v + 3 + c] = u + h;
      }
      if (bad_any) atomicAdd(&cnt->nonfinite, 1ull);
    }
    const int64_t slot0 = ves_patch_off[v];
    if (!bad_any)
      for (int k = threadIdx.x; k < np; k += blockDim.x)
        for (int c = 0; c < 3; ++c) {
          patch_box[6 * (slot0 + k) + c] = okey_inv(pk[k][c]) - h;
          patch_box[6 * (slot0 + k) + 3 + c] = okey_inv(pk[k][3 + c]) + h;
        }
    __syncthreads();
  }
}

// Per vesicle: the number of patches of its topology and its scene index.
__global__ void k_ves_tables(DevScene S, DevTopo T, int64_t *patch_cnt, int *ves_scene) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < S.n_ves; v += gridDim.x * blockDim.x) {
    const int t = S.topo_id[v];
    patch_cnt[v] = T.patch_off[t + 1] - T.patch_off[t];
    int lo = 0, hi = S.n_scenes;  // invariant: scene_off[lo] <= v < scene_off[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (S.scene_off[mid] <= v) lo = mid; else hi = mid;
    }
    ves_scene[v] = lo;
  }
}

}  // namespace

void launch_boxes(const DevScene &S, const DevTopo &T, double h, const int64_t *ves_patch_off, double *ves_box,
                  double *patch_box, int max_patches, Counters *cnt, hipStream_t st) {
  int g = S.n_ves < 8192 ? S.n_ves : 8192;
  if (g < 1) return;
  if (max_patches <= 128)
    k_boxes<128><<<g, 256, 0, st>>>(S, T, h, ves_patch_off, ves_box, patch_box, cnt);
  else if (max_patches <= 512)
    k_boxes<512><<<g, 256, 0, st>>>(S, T, h, ves_patch_off, ves_box, patch_box, cnt);
  else
    k_boxes<kMaxPatchesPerVes><<<g, 256, 0, st>>>(S, T, h, ves_patch_off, ves_box, patch_box, cnt);
}

void launch_ves_tables(const DevScene &S, const DevTopo &T, int64_t *patch_cnt, int *ves_scene, hipStream_t st) {
  int g = (S.n_ves + 255) / 256;
  if (g < 1) return;
  if (g > 1024) g = 1024;
  k_ves_tables<<<g, 256, 0, st>>>(S, T, patch_cnt, ves_scene);
}

}  // namespace stiv
