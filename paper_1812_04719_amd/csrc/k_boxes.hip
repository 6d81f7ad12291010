// K0: space-time bounding boxes (Sec. 3.3.1; Alg. 2, getBoundingBox).
//
// A vesicle's box is the componentwise min/max over all its vertices at t_n
// and t_{n+1}, inflated by h = d/2 per side.  min/max are exact, so the
// FP64 box is bit-identical to any other correct evaluation.  Patch boxes
// (the same over the vertices referenced by a patch's triangles) feed the
// primitive broad phase.  One workgroup streams one vesicle's SoA positions
// with coalesced 8-byte lanes; this is the one stage that reads every byte
// of X0 and X1.
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

__global__ __launch_bounds__(256) void k_boxes(DevScene S, DevTopo T, double h, const int64_t *ves_patch_off,
                                               double *ves_box, double *patch_box, Counters *cnt) {
  __shared__ double red[4][6];
  __shared__ int bad_any;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t nv_all = S.n_vtx;
  for (int v = blockIdx.x; v < S.n_ves; v += gridDim.x) {
    const int base = S.vtx_off[v];
    const int nvv = S.vtx_off[v + 1] - base;
    double lo[3], hi[3];
    for (int c = 0; c < 3; ++c) { lo[c] = INFINITY; hi[c] = -INFINITY; }
    int bad = 0;
    if (threadIdx.x == 0) bad_any = 0;
    for (int i = threadIdx.x; i < nvv; i += blockDim.x) {
      for (int c = 0; c < 3; ++c) {
        double a = S.x0[c * nv_all + base + i], b = S.x1[c * nv_all + base + i];
        bad |= !(isfinite(a) && isfinite(b));
        lo[c] = fmin(lo[c], fmin(a, b));
        hi[c] = fmax(hi[c], fmax(a, b));
      }
    }
    for (int c = 0; c < 3; ++c) {
      lo[c] = wave_min(lo[c]);
      hi[c] = wave_max(hi[c]);
    }
    if (lane == 0)
      for (int c = 0; c < 3; ++c) { red[wave][c] = lo[c]; red[wave][3 + c] = hi[c]; }
    __syncthreads();
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
    // patch boxes: one wave per patch
    const int t = S.topo_id[v];
    const int p0 = T.patch_off[t], p1 = T.patch_off[t + 1];
    const int64_t slot0 = ves_patch_off[v];
    for (int k = wave; k < p1 - p0; k += 4) {
      const int P = p0 + k;
      double pl[3], ph[3];
      for (int c = 0; c < 3; ++c) { pl[c] = INFINITY; ph[c] = -INFINITY; }
      for (int r = T.pref_off[P] + lane; r < T.pref_off[P + 1]; r += 64) {
        const int64_t g = base + T.pref[r];
        for (int c = 0; c < 3; ++c) {
          double a = S.x0[c * nv_all + g], b = S.x1[c * nv_all + g];
          pl[c] = fmin(pl[c], fmin(a, b));
          ph[c] = fmax(ph[c], fmax(a, b));
        }
      }
      for (int c = 0; c < 3; ++c) {
        pl[c] = wave_min(pl[c]);
        ph[c] = wave_max(ph[c]);
      }
      if (lane == 0)
        for (int c = 0; c < 3; ++c) {
          patch_box[6 * (slot0 + k) + c] = pl[c] - h;
          patch_box[6 * (slot0 + k) + 3 + c] = ph[c] + h;
        }
    }
    __syncthreads();
  }
}

__global__ void k_ves_patch_count(DevScene S, DevTopo T, int64_t *out) {
  for (int v = blockIdx.x * blockDim.x + threadIdx.x; v < S.n_ves; v += gridDim.x * blockDim.x) {
    const int t = S.topo_id[v];
    out[v] = T.patch_off[t + 1] - T.patch_off[t];
  }
}

}  // namespace

void launch_boxes(const DevScene &S, const DevTopo &T, double h, const int64_t *ves_patch_off, double *ves_box,
                  double *patch_box, Counters *cnt, hipStream_t st) {
  int g = S.n_ves < 8192 ? S.n_ves : 8192;
  if (g < 1) return;
  k_boxes<<<g, 256, 0, st>>>(S, T, h, ves_patch_off, ves_box, patch_box, cnt);
}

void launch_ves_patch_count(const DevScene &S, const DevTopo &T, int64_t *out, hipStream_t st) {
  int g = (S.n_ves + 255) / 256;
  if (g < 1) return;
  if (g > 1024) g = 1024;
  k_ves_patch_count<<<g, 256, 0, st>>>(S, T, out);
}

}  // namespace stiv
