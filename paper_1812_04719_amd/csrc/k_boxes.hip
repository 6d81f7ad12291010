// K0: space-time bounding boxes (Sec. 3.3.1; Alg. 2, getBoundingBox).
//
// A vesicle's box is the componentwise min/max over all its vertices at t_n
// and t_{n+1}, inflated by h = d/2 per side.  min/max are exact, so the
// FP64 box is bit-identical to any other correct evaluation.  Patch boxes
// (the same over the vertices referenced by a patch's triangles) feed the
// primitive broad phase.  One workgroup streams one vesicle's SoA positions
// with coalesced 8-byte lanes, once; this is the one stage that reads every
// byte of X0 and X1.
#include <hip/hip_fp16.h>

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
// are not extreme, and neighbouring lanes often hit the same patch).  Any
// earlier value is looser than the current one, so the six reads are plain
// loads, which the compiler may pair into wider ones.
__device__ inline void fold_box(unsigned long long (*pk)[6], int q, const unsigned long long kl[3],
                                const unsigned long long ku[3]) {
  unsigned long long cur[6];
#pragma unroll
  for (int c = 0; c < 6; ++c) cur[c] = pk[q][c];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (kl[c] < cur[c]) atomicMin(&pk[q][c], kl[c]);
    if (ku[c] > cur[3 + c]) atomicMax(&pk[q][3 + c], ku[c]);
  }
}

// Order-preserving map of floats to unsigned 32-bit keys (finite or infinite).
__device__ inline unsigned int fkey(float x) {
  const unsigned int b = __float_as_uint(x);
  return (b >> 31) ? ~b : (b | 0x80000000u);
}
__device__ inline float fkey_inv(unsigned int k) {
  const unsigned int b = (k >> 31) ? (k & 0x7fffffffu) : ~k;
  return __uint_as_float(b);
}

// FP32 values at or below (above) x: the nearest float moved down (up) by
// 2^-22 of its magnitude, at least two units in its last place (plus 1e-30
// for values near zero); cheaper than a conversion with a directed rounding
// mode.
__device__ inline float f32_below(double x) {
  const float f = (float)x;
  return f - (fabsf(f) * 2.384185791015625e-07f + 1e-30f);
}
__device__ inline float f32_above(double x) {
  const float f = (float)x;
  return f + (fabsf(f) * 2.384185791015625e-07f + 1e-30f);
}

// Lower and upper support of the box anchor + [lo, hi] along the six face
// diagonals, in FP64 and rounded outward to FP32.
__device__ inline void dop_support(const float lo[3], const float hi[3], const double an[3], float out[kDopVals]) {
  const double lx = lo[0], ly = lo[1], lz = lo[2], hx = hi[0], hy = hi[1], hz = hi[2];
  const double axy = an[0] + an[1], axmy = an[0] - an[1], axz = an[0] + an[2], axmz = an[0] - an[2],
               ayz = an[1] + an[2], aymz = an[1] - an[2];
  const double dn[kDopDirs] = {(lx + ly) + axy, (lx - hy) + axmy, (lx + lz) + axz,
                               (lx - hz) + axmz, (ly + lz) + ayz, (ly - hz) + aymz};
  const double up[kDopDirs] = {(hx + hy) + axy, (hx - ly) + axmy, (hx + hz) + axz,
                               (hx - lz) + axmz, (hy + hz) + ayz, (hy - lz) + aymz};
#pragma unroll
  for (int j = 0; j < kDopDirs; ++j) {
    out[2 * j] = f32_below(dn[j]);
    out[2 * j + 1] = f32_above(up[j]);
  }
}

// Supports of a triangle's box, the union of its vertices' boxes: rows of
// vb (indexed by local vertex id) hold each vertex's box relative to the
// vesicle's anchor in FP16, rounded outward, as three half pairs (lo x, lo y),
// (lo z, hi x), (hi y, hi z).
__device__ inline void tri_support(const unsigned int *vb, int4 rec, const double an[3], float sp[kDopVals]) {
  float v[3][6];
  const int ids[3] = {rec.x, rec.y, rec.z};
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int w = 0; w < 3; ++w) {
      const unsigned int u = vb[3 * ids[k] + w];
      v[k][2 * w] = __half2float(__ushort_as_half((unsigned short)(u & 0xffffu)));
      v[k][2 * w + 1] = __half2float(__ushort_as_half((unsigned short)(u >> 16)));
    }
  float tl[3], th[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    tl[c] = fminf(fminf(v[0][c], v[1][c]), v[2][c]);
    th[c] = fmaxf(fmaxf(v[0][3 + c], v[1][3 + c]), v[2][3 + c]);
  }
  dop_support(tl, th, an, sp);
}

// One workgroup per vesicle: each thread streams vertices (coalesced SoA
// loads of X0 and X1), folds them into the vesicle box and, through the
// vertex -> patch incidence (packed four to a vertex), into the LDS boxes of
// the patches that reference the vertex.  With `dop`, each vertex's
// space-time box is also kept in LDS, relative to the vesicle's first vertex
// in FP16 rounded outward (an offset wider than FP16's range becomes
// infinite, which only loosens the bound), and a second pass forms every
// patch's supports along the face diagonals from its triangles' boxes (the
// union of their vertices' boxes).  The patch's 9-DOP (its box
// and these supports) contains the boxes of all its primitives, since every
// owned vertex and edge lies in one of its triangles: two patches whose
// supports do not meet along some diagonal hold no primitive pair with
// meeting boxes.
// The two parts can run as two launches (the boxes, then the supports, which
// read the positions again), so that the supports overlap the vesicle broad
// phase, which needs only the vesicle boxes.
// MAXP bounds the patches of any vesicle's topology (LDS is sized for it, so
// small meshes keep more workgroups resident); PARTS selects the parts.
constexpr int kBoxU = 4;
constexpr int kTriPerThread = 4;

template <int MAXP, int PARTS>
__global__ __launch_bounds__(256) void k_boxes(DevScene S, DevTopo T, double h, const int64_t *ves_patch_off,
                                               double *ves_box, double *patch_box, float *patch_dop, Counters *cnt) {
  // boxes: vesicle and patch boxes; dop: the supports (FP16 vertex boxes and
  // their folding)
  constexpr bool boxes = PARTS & kBoxParts, dop = PARTS & kSupportParts;
  __shared__ unsigned long long pk[MAXP][6];  // lo as key, hi as key
  constexpr int kDopP = MAXP <= 512 ? MAXP : 1;  // supports for meshes of up to 512 patches
  __shared__ unsigned int dk[kDopP][kDopVals];   // the patches' supports as keys
  extern __shared__ unsigned int vbox[];  // with dop: [n_vertices][3] half pairs, each vertex's box (tri_support)
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
    // anchor of the FP16 vertex boxes: the vesicle's first vertex at t_n
    const double an[3] = {S.x0[base], S.x0[nv_all + base], S.x0[2 * nv_all + base]};
    for (int k = threadIdx.x; k < np; k += blockDim.x) {
      if (boxes)
        for (int c = 0; c < 3; ++c) { pk[k][c] = ~0ull; pk[k][3 + c] = 0ull; }
      if (dop)
        for (int j = 0; j < kDopDirs; ++j) { dk[k][2 * j] = ~0u; dk[k][2 * j + 1] = 0u; }
    }
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
        q4[k] = (in && boxes) ? T.vp4[vb + i] : make_int4(-1, -1, -1, -1);
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
        if (dop) {
          // the vertex box relative to the anchor, rounded outward to FP16
          unsigned short hv[6];
#pragma unroll
          for (int c = 0; c < 3; ++c) {
            hv[c] = __half_as_ushort(__float2half_rd(f32_below((l[c] - h) - an[c])));
            hv[3 + c] = __half_as_ushort(__float2half_ru(f32_above((u[c] + h) - an[c])));
          }
#pragma unroll
          for (int w = 0; w < 3; ++w) vbox[3 * i + w] = (unsigned int)hv[2 * w] | ((unsigned int)hv[2 * w + 1] << 16);
        }
        if (!boxes) continue;
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
    if (dop) {
      // face-diagonal supports of each patch: the vesicle's triangles in patch
      // order, kTriPerThread consecutive ones per thread (mostly of one patch:
      // kept in registers, folded into the patch's LDS supports once per run)
      __syncthreads();
      const int pt0 = T.patch_off[t];
      const int r_beg = T.ptri_off[pt0], r_end = T.ptri_off[pt0 + np];
      for (int r0 = r_beg + kTriPerThread * threadIdx.x; r0 < r_end; r0 += kTriPerThread * blockDim.x) {
        int4 rec[kTriPerThread];
#pragma unroll
        for (int u = 0; u < kTriPerThread; ++u) rec[u] = r0 + u < r_end ? T.tri_rec[r0 + u] : make_int4(0, 0, 0, -1);
        float acc[kDopVals];
        int cur = rec[0].w;
#pragma unroll
        for (int j = 0; j < kDopDirs; ++j) { acc[2 * j] = INFINITY; acc[2 * j + 1] = -INFINITY; }
#pragma unroll
        for (int u = 0; u <= kTriPerThread; ++u) {
          const int pu = u < kTriPerThread ? rec[u].w : -1;
          if (pu != cur) {  // end of a run of one patch: fold it (skipping what cannot improve)
#pragma unroll
            for (int j = 0; j < kDopDirs; ++j) {
              // plain reads: an earlier value is looser (see fold_box)
              const unsigned int kd = fkey(acc[2 * j]), ku = fkey(acc[2 * j + 1]);
              const unsigned int cd = dk[cur][2 * j], cu = dk[cur][2 * j + 1];
              if (kd < cd) atomicMin(&dk[cur][2 * j], kd);
              if (ku > cu) atomicMax(&dk[cur][2 * j + 1], ku);
              acc[2 * j] = INFINITY;
              acc[2 * j + 1] = -INFINITY;
            }
            cur = pu;
          }
          if (pu < 0) break;
          float sp[kDopVals];
          tri_support(vbox, rec[u], an, sp);
#pragma unroll
          for (int j = 0; j < kDopDirs; ++j) {
            acc[2 * j] = fminf(acc[2 * j], sp[2 * j]);
            acc[2 * j + 1] = fmaxf(acc[2 * j + 1], sp[2 * j + 1]);
          }
        }
      }
    }
    if (!boxes) {
      // the supports alone
      __syncthreads();
      const int64_t slot0 = ves_patch_off[v];
      for (int k = threadIdx.x; k < np; k += blockDim.x)
        for (int j = 0; j < kDopVals; ++j) patch_dop[kDopVals * (slot0 + k) + j] = fkey_inv(dk[k][j]);
      __syncthreads();
      continue;
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
      for (int k = threadIdx.x; k < np; k += blockDim.x) {
        for (int c = 0; c < 3; ++c) {
          patch_box[6 * (slot0 + k) + c] = okey_inv(pk[k][c]) - h;
          patch_box[6 * (slot0 + k) + 3 + c] = okey_inv(pk[k][3 + c]) + h;
        }
        if (dop)
          for (int j = 0; j < kDopVals; ++j) patch_dop[kDopVals * (slot0 + k) + j] = fkey_inv(dk[k][j]);
        else if (PARTS & kNoSupportParts)
          for (int j = 0; j < kDopVals; ++j) patch_dop[kDopVals * (slot0 + k) + j] = (j & 1) ? INFINITY : -INFINITY;
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



// The same tables for up to kVesTablesOne vesicles in one workgroup, which
// also scans the patch counts into the vesicles' first patch slots
// (patch_off[n] = all slots): one launch instead of two.
constexpr int kVesTablesOne = 8192;
__global__ __launch_bounds__(1024) void k_ves_tables_one(DevScene S, DevTopo T, int64_t *patch_cnt, int *ves_scene,
                                                         int64_t *patch_off) {
  __shared__ int64_t sh_wave[16];
  const int n = S.n_ves;
  const int chunk = (n + 1023) / 1024;
  const int lo = (int)threadIdx.x * chunk, hi = lo + chunk < n ? lo + chunk : n;
  int64_t run = 0;
  for (int v = lo; v < hi; ++v) {
    const int t = S.topo_id[v];
    const int64_t c = T.patch_off[t + 1] - T.patch_off[t];
    patch_cnt[v] = c;
    run += c;
    int a = 0, b = S.n_scenes;  // invariant: scene_off[a] <= v < scene_off[b]
    while (b - a > 1) {
      const int mid = (a + b) >> 1;
      if (S.scene_off[mid] <= v) a = mid; else b = mid;
    }
    ves_scene[v] = a;
  }
  // exclusive scan of the runs: shuffles within each wavefront, then the
  // totals of the wavefronts before it
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  int64_t incl = run;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int64_t y = __shfl_up(incl, o, 64);
    if (lane >= o) incl += y;
  }
  if (lane == 63) sh_wave[wave] = incl;
  __syncthreads();
  for (int w = 0; w < wave; ++w) incl += sh_wave[w];
  int64_t at = incl - run;
  for (int v = lo; v < hi; ++v) {
    patch_off[v] = at;
    at += patch_cnt[v];
  }
  if (threadIdx.x == 1023) patch_off[n] = incl;
}

}  // namespace

// The FP16 vertex boxes for the patch supports (12 bytes per vertex) fit in
// LDS up to this many vertices per mesh (order-32 meshes have 2114, order 44
// 3962); meshes of more vertices or
// more than 512 patches keep the axis-aligned patch boxes alone (their
// supports are written as -inf, +inf, which never cull).
constexpr int kDopMaxVertices = 4096;

bool boxes_have_supports(const DevTopo &T, int max_patches) {
  return T.tri_rec != nullptr && T.max_nv <= kDopMaxVertices && max_patches <= 512;
}

template <int PARTS>
static void launch_parts(const DevScene &S, const DevTopo &T, double h, const int64_t *ves_patch_off,
                         double *ves_box, double *patch_box, float *patch_dop, int max_patches, int grid_max,
                         Counters *cnt, hipStream_t st) {
  const int g = S.n_ves < grid_max ? S.n_ves : grid_max;
  const size_t lds = (PARTS & kSupportParts) ? sizeof(unsigned int) * 3 * (size_t)T.max_nv : 0;
  if (max_patches <= 128)
    k_boxes<128, PARTS><<<g, 256, lds, st>>>(S, T, h, ves_patch_off, ves_box, patch_box, patch_dop, cnt);
  else if (max_patches <= 512)
    k_boxes<512, PARTS><<<g, 256, lds, st>>>(S, T, h, ves_patch_off, ves_box, patch_box, patch_dop, cnt);
  else
    k_boxes<kMaxPatchesPerVes, PARTS><<<g, 256, lds, st>>>(S, T, h, ves_patch_off, ves_box, patch_box, patch_dop, cnt);
}

void launch_boxes(const DevScene &S, const DevTopo &T, double h, const int64_t *ves_patch_off, double *ves_box,
                  double *patch_box, float *patch_dop, int max_patches, int parts, int grid_max, Counters *cnt,
                  hipStream_t st) {
  if (S.n_ves < 1) return;
  if (parts == kBoxParts)
    launch_parts<kBoxParts>(S, T, h, ves_patch_off, ves_box, patch_box, patch_dop, max_patches, grid_max, cnt, st);
  else if (parts == kSupportParts)
    launch_parts<kSupportParts>(S, T, h, ves_patch_off, ves_box, patch_box, patch_dop, max_patches, grid_max, cnt,
                                st);
  else if (parts == (kBoxParts | kSupportParts))
    launch_parts<kBoxParts | kSupportParts>(S, T, h, ves_patch_off, ves_box, patch_box, patch_dop, max_patches,
                                            grid_max, cnt, st);
  else
    launch_parts<kBoxParts | kNoSupportParts>(S, T, h, ves_patch_off, ves_box, patch_box, patch_dop, max_patches,
                                              grid_max, cnt, st);
}

bool launch_ves_tables(const DevScene &S, const DevTopo &T, int64_t *patch_cnt, int *ves_scene, int64_t *patch_off,
                       hipStream_t st) {
  if (S.n_ves <= kVesTablesOne) {
    k_ves_tables_one<<<1, 1024, 0, st>>>(S, T, patch_cnt, ves_scene, patch_off);
    return true;
  }
  int g = (S.n_ves + 255) / 256;
  if (g > 1024) g = 1024;
  k_ves_tables<<<g, 256, 0, st>>>(S, T, patch_cnt, ves_scene);
  return false;
}

}  // namespace stiv
