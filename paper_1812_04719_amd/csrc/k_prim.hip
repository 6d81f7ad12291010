// K2: primitive broad phase inside each candidate vesicle pair.
//
// A primitive's space-time box is the min/max of its 1, 2 or 3 vertices at
// both times, inflated by h = d/2 and shifted by the pair's image shift
// (same arithmetic, same order as the vesicle boxes, so the closed-interval
// FP64 test is exact).  Candidates are vertex-triangle pairs in both
// directions and edge-edge pairs whose boxes intersect (Sec. 3.3.2,
// checkContact of Alg. 2 works on exactly these primitives of a pair).
//
// Two kernels:
//   k_patch_pairs  one workgroup per vesicle pair: cull each side's patches
//                  against the other vesicle's box, then test the surviving
//                  patch pairs; emit (pair, patch a, patch b) work items.
//   k_prim_cand    one wavefront per work item: stage the two patches'
//                  per-vertex boxes in LDS (FP32, rounded outward), cull each
//                  primitive against the other patch's box, then each lane
//                  holds one left-hand primitive box in registers and sweeps
//                  the right-hand list from LDS; hits are buffered in LDS and
//                  flushed with one atomic per batch.
#include "stiv_common.h"

namespace stiv {

namespace {

__device__ inline bool ov6(const double *A, const double *B) {
  return A[0] <= B[3] && B[0] <= A[3] && A[1] <= B[4] && B[1] <= A[4] && A[2] <= B[5] && B[2] <= A[5];
}

__device__ inline unsigned long long lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Wavefront-aggregated append: returns this lane's slot (valid iff `want`).
__device__ inline unsigned long long wave_append(bool want, unsigned long long *counter) {
  const unsigned long long m = __ballot(want);
  const int n = __popcll(m);
  unsigned long long base = 0;
  const int leader = m ? __ffsll((long long)m) - 1 : 0;
  if ((int)(threadIdx.x & 63) == leader && n) base = atomicAdd(counter, (unsigned long long)n);
  base = __shfl(base, leader, 64);
  return base + __popcll(m & lanemask_lt());
}

constexpr int kPPThreads = 256;

__global__ __launch_bounds__(kPPThreads) void k_patch_pairs(DevScene S, DevTopo T, const PairRec *pairs,
                                                            const double *ves_box, const int64_t *ves_patch_off,
                                                            const double *patch_box, uint64_t *work,
                                                            int64_t work_cap, Counters *cnt, int64_t pairs_cap) {
  __shared__ int sA[kMaxPatchesPerVes], sB[kMaxPatchesPerVes];
  __shared__ int nA, nB;
  int64_t np = (int64_t)cnt->n_pairs;
  np = np < pairs_cap ? np : pairs_cap;
  for (int64_t p = blockIdx.x; p < np; p += gridDim.x) {
    const PairRec pr = pairs[p];
    double boxA[6], boxB[6];
    for (int c = 0; c < 6; ++c) boxA[c] = ves_box[6 * (int64_t)pr.a + c];
    for (int c = 0; c < 3; ++c) {
      boxB[c] = ves_box[6 * (int64_t)pr.b + c] + pr.sh[c];
      boxB[3 + c] = ves_box[6 * (int64_t)pr.b + 3 + c] + pr.sh[c];
    }
    const int64_t pa0 = ves_patch_off[pr.a], pb0 = ves_patch_off[pr.b];
    const int na = (int)(ves_patch_off[pr.a + 1] - pa0), nb = (int)(ves_patch_off[pr.b + 1] - pb0);
    if (threadIdx.x == 0) { nA = 0; nB = 0; }
    __syncthreads();
    for (int k = threadIdx.x; k < na; k += blockDim.x) {
      const double *P = patch_box + 6 * (pa0 + k);
      if (ov6(P, boxB)) sA[atomicAdd(&nA, 1)] = k;
    }
    for (int k = threadIdx.x; k < nb; k += blockDim.x) {
      const double *P = patch_box + 6 * (pb0 + k);
      double Q[6];
      for (int c = 0; c < 3; ++c) { Q[c] = P[c] + pr.sh[c]; Q[3 + c] = P[3 + c] + pr.sh[c]; }
      if (ov6(Q, boxA)) sB[atomicAdd(&nB, 1)] = k;
    }
    __syncthreads();
    const int ma = nA, mb = nB;
    const int tot = ma * mb;
    for (int base = 0; base < tot; base += blockDim.x) {
      const int t = base + threadIdx.x;
      bool hit = false;
      int ia = 0, ib = 0;
      if (t < tot) {
        ia = sA[t / mb];
        ib = sB[t % mb];
        const double *P = patch_box + 6 * (pa0 + ia);
        const double *Qr = patch_box + 6 * (pb0 + ib);
        double Q[6];
        for (int c = 0; c < 3; ++c) { Q[c] = Qr[c] + pr.sh[c]; Q[3 + c] = Qr[3 + c] + pr.sh[c]; }
        hit = ov6(P, Q);
      }
      const unsigned long long slot = wave_append(hit, &cnt->n_work);
      if (hit && (int64_t)slot < work_cap)
        work[slot] = ((uint64_t)p << 32) | ((uint64_t)ia << 16) | (uint64_t)ib;
    }
    __syncthreads();
  }
}

// --------------------------------------------------------------------------
// Per work item: one wavefront.
//
// The primitive boxes here are FP32, rounded outward from the FP64 boxes, so
// every pair whose FP64 boxes intersect passes (a superset).  The exact FP64
// test is made by the narrow-phase kernel, which loads the same four vertices
// anyway; only pairs passing it count as candidates.
// --------------------------------------------------------------------------
constexpr int kHitBuf = 256;

struct WaveLds {
  float vb[2][kMaxPatchRef][6];  // per-vertex boxes: ((min - h) + sh, (max + h) + sh), outward to FP32
  float rbox[kMaxPatchOwnE][6];  // right-hand list (current kind): boxes
  int rid[kMaxPatchOwnE];        //   and primitive ids
  int lk[kMaxPatchOwnE];         // left-hand list: patch-table index of the primitive
  int nl, nr, nh;
  Cand hits[kHitBuf];
};

__device__ inline bool ov6f(const float *A, const float *B) {
  return A[0] <= B[3] && B[0] <= A[3] && A[1] <= B[4] && B[1] <= A[4] && A[2] <= B[5] && B[2] <= A[5];
}

__device__ inline void box_from_slots(const float (*vb)[6], const uint8_t *slot, int nvert, float *out) {
  for (int c = 0; c < 6; ++c) out[c] = vb[slot[0]][c];
  for (int k = 1; k < nvert; ++k)
    for (int c = 0; c < 3; ++c) {
      out[c] = fminf(out[c], vb[slot[k]][c]);
      out[3 + c] = fmaxf(out[3 + c], vb[slot[k]][3 + c]);
    }
}

__device__ inline float wave_minf(float v) {
  for (int off = 32; off > 0; off >>= 1) v = fminf(v, __shfl_xor(v, off, 64));
  return v;
}
__device__ inline float wave_maxf(float v) {
  for (int off = 32; off > 0; off >>= 1) v = fmaxf(v, __shfl_xor(v, off, 64));
  return v;
}

// Move the wave's buffered hits to the global pre-candidate list.
__device__ inline void flush_hits(WaveLds &W, Cand *out, int64_t cap, unsigned long long *counter) {
  const int lane = threadIdx.x;
  const int n = W.nh;
  unsigned long long base = 0;
  if (lane == 0 && n) base = atomicAdd(counter, (unsigned long long)n);
  base = __shfl(base, 0, 64);
  for (int k = lane; k < n; k += 64)
    if ((int64_t)(base + k) < cap) out[base + k] = W.hits[k];
  __syncthreads();
  if (lane == 0) W.nh = 0;
  __syncthreads();
}

__global__ __launch_bounds__(64) void k_prim_cand(DevScene S, DevTopo T, const PairRec *pairs,
                                                  const int64_t *ves_patch_off, const double *patch_box,
                                                  const uint64_t *work, int64_t work_cap, double h, Cand *cand,
                                                  int64_t cand_cap, Counters *cnt) {
  __shared__ WaveLds W;
  const int lane = threadIdx.x;
  int64_t nw = (int64_t)cnt->n_work;
  nw = nw < work_cap ? nw : work_cap;
  if (lane == 0) W.nh = 0;
  __syncthreads();
  for (int64_t w = blockIdx.x; w < nw; w += gridDim.x) {
    const uint64_t wr = work[w];
    const int p = (int)(wr >> 32);
    const int pk[2] = {(int)((wr >> 16) & 0xffffu), (int)(wr & 0xffffu)};
    const PairRec pr = pairs[p];
    const int ves[2] = {pr.a, pr.b};
    int P[2];
    float pb[2][6];
    for (int side = 0; side < 2; ++side) {
      P[side] = T.patch_off[S.topo_id[ves[side]]] + pk[side];
      const int base = S.vtx_off[ves[side]];
      const int r0 = T.pref_off[P[side]], nref = T.pref_off[P[side] + 1] - r0;
      const double sh[3] = {side ? pr.sh[0] : 0.0, side ? pr.sh[1] : 0.0, side ? pr.sh[2] : 0.0};
      float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
      for (int r = lane; r < nref; r += 64) {
        const int64_t g = base + T.pref[r0 + r];
        for (int c = 0; c < 3; ++c) {
          const double a = S.x0[c * (int64_t)S.n_vtx + g], b = S.x1[c * (int64_t)S.n_vtx + g];
          const float l = __double2float_rd((fmin(a, b) - h) + sh[c]);
          const float u = __double2float_ru((fmax(a, b) + h) + sh[c]);
          W.vb[side][r][c] = l;
          W.vb[side][r][3 + c] = u;
          lo[c] = fminf(lo[c], l);
          hi[c] = fmaxf(hi[c], u);
        }
      }
      for (int c = 0; c < 3; ++c) {
        pb[side][c] = wave_minf(lo[c]);
        pb[side][3 + c] = wave_maxf(hi[c]);
      }
    }
    __syncthreads();
    for (int kind = 0; kind < 3; ++kind) {
      const int sl = (kind == 1) ? 1 : 0, sr = 1 - sl;
      // left list: owned vertices (kinds 0, 1) or owned edges (kind 2) of side sl
      const int lbeg = kind == 2 ? T.pedge_off[P[sl]] : T.pvtx_off[P[sl]];
      const int lend = kind == 2 ? T.pedge_off[P[sl] + 1] : T.pvtx_off[P[sl] + 1];
      const uint8_t *lslot = kind == 2 ? T.pedge_slot : T.pvtx_slot;
      const int lnv = kind == 2 ? 2 : 1;
      // right list: triangles (kinds 0, 1) or owned edges (kind 2) of side sr
      const int rbeg = kind == 2 ? T.pedge_off[P[sr]] : T.ptri_off[P[sr]];
      const int rend = kind == 2 ? T.pedge_off[P[sr] + 1] : T.ptri_off[P[sr] + 1];
      const uint8_t *rslot = kind == 2 ? T.pedge_slot : T.ptri_slot;
      const int *rids = kind == 2 ? T.pedge : T.ptri;
      const int rnv = kind == 2 ? 2 : 3;
      if (lane == 0) { W.nl = 0; W.nr = 0; }
      __syncthreads();
      for (int k = lbeg + lane; k < lend; k += 64) {
        float bx[6];
        box_from_slots(W.vb[sl], lslot + (int64_t)lnv * k, lnv, bx);
        if (ov6f(bx, pb[sr])) W.lk[atomicAdd(&W.nl, 1)] = k;
      }
      for (int k = rbeg + lane; k < rend; k += 64) {
        float bx[6];
        box_from_slots(W.vb[sr], rslot + (int64_t)rnv * k, rnv, bx);
        if (ov6f(bx, pb[sl])) {
          const int q = atomicAdd(&W.nr, 1);
          for (int c = 0; c < 6; ++c) W.rbox[q][c] = bx[c];
          W.rid[q] = rids[k];
        }
      }
      __syncthreads();
      const int nl = W.nl, nr = W.nr;
      const int *lids = kind == 2 ? T.pedge : T.pvtx;
      for (int l0 = 0; l0 < nl; l0 += 64) {
        const bool act = l0 + lane < nl;
        float lb[6];
        int lidv = 0;
        if (act) {
          const int k = W.lk[l0 + lane];
          box_from_slots(W.vb[sl], lslot + (int64_t)lnv * k, lnv, lb);
          lidv = lids[k];
        }
        for (int j = 0; j < nr; ++j) {
          if (*(volatile int *)&W.nh > kHitBuf - 64) flush_hits(W, cand, cand_cap, &cnt->n_pre);
          if (act && ov6f(lb, W.rbox[j])) {
            const int q = atomicAdd(&W.nh, 1);
            Cand cd;
            cd.pair = p; cd.kind = kind; cd.i = lidv; cd.j = W.rid[j];
            W.hits[q] = cd;
          }
        }
      }
      __syncthreads();
    }
  }
  flush_hits(W, cand, cand_cap, &cnt->n_pre);
}

}  // namespace

void launch_patch_pairs(const DevScene &S, const DevTopo &T, const PairRec *pairs, int64_t pairs_cap,
                        const double *ves_box, const int64_t *ves_patch_off, const double *patch_box,
                        uint64_t *work, int64_t work_cap, Counters *cnt, hipStream_t st) {
  k_patch_pairs<<<2048, kPPThreads, 0, st>>>(S, T, pairs, ves_box, ves_patch_off, patch_box, work, work_cap, cnt,
                                             pairs_cap);
}

void launch_prim_cand(const DevScene &S, const DevTopo &T, const PairRec *pairs, const int64_t *ves_patch_off,
                      const double *patch_box, const uint64_t *work, int64_t work_cap, double h, Cand *cand,
                      int64_t cand_cap, Counters *cnt, hipStream_t st) {
  k_prim_cand<<<8192, 64, 0, st>>>(S, T, pairs, ves_patch_off, patch_box, work, work_cap, h, cand, cand_cap, cnt);
}

}  // namespace stiv
