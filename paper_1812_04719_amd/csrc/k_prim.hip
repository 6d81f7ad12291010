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
//                  vertex boxes in LDS, cull each primitive against the other
//                  patch's box, test the survivors pairwise and compact the
//                  hits with a wavefront ballot + prefix count, one atomic per
//                  wavefront per batch.
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
// --------------------------------------------------------------------------
struct PrimList {
  double box[kMaxPatchOwnE][6];
  int id[kMaxPatchOwnE];
};

struct WaveLds {
  double vb[2][kMaxPatchRef][6];  // raw vertex boxes: min/max of X0, X1 (no inflation, no shift)
  PrimList L[2];
  int n[2];
};

// Box of a primitive from its vertex slots: (min - h) + sh, (max + h) + sh.
__device__ inline void prim_box(const double (*vb)[6], const uint8_t *slot, int nvert, double h,
                                const double *sh, double *out) {
  double lo[3], hi[3];
  for (int c = 0; c < 3; ++c) { lo[c] = vb[slot[0]][c]; hi[c] = vb[slot[0]][3 + c]; }
  for (int k = 1; k < nvert; ++k)
    for (int c = 0; c < 3; ++c) {
      lo[c] = fmin(lo[c], vb[slot[k]][c]);
      hi[c] = fmax(hi[c], vb[slot[k]][3 + c]);
    }
  for (int c = 0; c < 3; ++c) {
    out[c] = (lo[c] - h) + sh[c];
    out[3 + c] = (hi[c] + h) + sh[c];
  }
}

__global__ __launch_bounds__(64) void k_prim_cand(DevScene S, DevTopo T, const PairRec *pairs,
                                                  const int64_t *ves_patch_off, const double *patch_box,
                                                  const uint64_t *work, int64_t work_cap, double h, Cand *cand,
                                                  int64_t cand_cap, Counters *cnt) {
  __shared__ WaveLds W;
  const int lane = threadIdx.x;
  int64_t nw = (int64_t)cnt->n_work;
  nw = nw < work_cap ? nw : work_cap;
  const double zero[3] = {0.0, 0.0, 0.0};
  for (int64_t w = blockIdx.x; w < nw; w += gridDim.x) {
    const uint64_t wr = work[w];
    const int p = (int)(wr >> 32);
    const int ia = (int)((wr >> 16) & 0xffffu), ib = (int)(wr & 0xffffu);
    const PairRec pr = pairs[p];
    const int ves[2] = {pr.a, pr.b};
    const int pk[2] = {ia, ib};
    int P[2];
    double pbox[2][6];
    for (int side = 0; side < 2; ++side) {
      const int t = S.topo_id[ves[side]];
      P[side] = T.patch_off[t] + pk[side];
      const double *src = patch_box + 6 * (ves_patch_off[ves[side]] + pk[side]);
      const double *sh = side ? pr.sh : zero;
      for (int c = 0; c < 3; ++c) { pbox[side][c] = src[c] + sh[c]; pbox[side][3 + c] = src[3 + c] + sh[c]; }
      const int base = S.vtx_off[ves[side]];
      const int r0 = T.pref_off[P[side]], r1 = T.pref_off[P[side] + 1];
      for (int r = r0 + lane; r < r1; r += 64) {
        const int64_t g = base + T.pref[r];
        for (int c = 0; c < 3; ++c) {
          const double a = S.x0[c * (int64_t)S.n_vtx + g], b = S.x1[c * (int64_t)S.n_vtx + g];
          W.vb[side][r - r0][c] = fmin(a, b);
          W.vb[side][r - r0][3 + c] = fmax(a, b);
        }
      }
    }
    __syncthreads();
    // three phases: kind 0 (vertices of a x triangles of b), kind 1 (vertices
    // of b x triangles of a), kind 2 (edges of a x edges of b)
    for (int kind = 0; kind < 3; ++kind) {
      // list 0: the "left" primitive (vertex or edge of side sl), list 1: triangle or edge of side sr
      const int sl = (kind == 1) ? 1 : 0;
      const int sr = 1 - sl;
      for (int li = 0; li < 2; ++li) {
        const int side = li == 0 ? sl : sr;
        const double *sh = side ? pr.sh : zero;
        const double *other = pbox[1 - side];
        int beg, end, nvert;
        const int *ids;
        const uint8_t *slots;
        if (kind == 2) {
          beg = T.pedge_off[P[side]]; end = T.pedge_off[P[side] + 1]; ids = T.pedge; slots = T.pedge_slot; nvert = 2;
        } else if (li == 0) {
          beg = T.pvtx_off[P[side]]; end = T.pvtx_off[P[side] + 1]; ids = T.pvtx; slots = T.pvtx_slot; nvert = 1;
        } else {
          beg = T.ptri_off[P[side]]; end = T.ptri_off[P[side] + 1]; ids = T.ptri; slots = T.ptri_slot; nvert = 3;
        }
        if (lane == 0) W.n[li] = 0;
        __syncthreads();
        for (int k0 = beg; k0 < end; k0 += 64) {
          const int k = k0 + lane;
          double bx[6];
          bool keep = false;
          if (k < end) {
            prim_box(W.vb[side], slots + (int64_t)nvert * k, nvert, h, sh, bx);
            keep = ov6(bx, other);
          }
          const unsigned long long m = __ballot(keep);
          const int pos = W.n[li] + __popcll(m & lanemask_lt());
          if (keep) {
            for (int c = 0; c < 6; ++c) W.L[li].box[pos][c] = bx[c];
            W.L[li].id[pos] = ids[k];
          }
          __syncthreads();
          if (lane == 0) W.n[li] += __popcll(m);
          __syncthreads();
        }
      }
      const int n0 = W.n[0], n1 = W.n[1];
      const int tot = n0 * n1;
      for (int base = 0; base < tot; base += 64) {
        const int t = base + lane;
        bool hit = false;
        int i = 0, j = 0;
        if (t < tot) {
          const int x = t / n1, y = t % n1;
          hit = ov6(W.L[0].box[x], W.L[1].box[y]);
          i = W.L[0].id[x];
          j = W.L[1].id[y];
        }
        const unsigned long long slot = wave_append(hit, &cnt->n_cand);
        const int nh = __popcll(__ballot(hit));
        if (lane == 0 && nh) atomicAdd(kind == 2 ? &cnt->n_cand_ee : &cnt->n_cand_vt, (unsigned long long)nh);
        if (hit && (int64_t)slot < cand_cap) {
          Cand cd;
          cd.pair = p; cd.kind = kind; cd.i = i; cd.j = j;
          cand[slot] = cd;
        }
      }
      __syncthreads();
    }
  }
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
