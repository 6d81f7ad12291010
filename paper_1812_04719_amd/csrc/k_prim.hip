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
//   k_prim_cand    one wavefront per work item: FP32 register-tiled filter
//                  over LDS-staged patches, then the exact FP64 box test and
//                  the polynomial screen of the narrow phase on the hits.
#include "narrow_math.h"

namespace stiv {

namespace {

__device__ inline bool ov6(const double *A, const double *B) {
  return A[0] <= B[3] && B[0] <= A[3] && A[1] <= B[4] && B[1] <= A[4] && A[2] <= B[5] && B[2] <= A[5];
}

__device__ inline unsigned long long lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

constexpr int kPPThreads = 256;
constexpr int kPPBuf = 512;

// Slot for each lane with take set in an LDS list whose length is *n: one
// atomic per wavefront, lanes in lane order.  Every lane of the wavefront
// must call it.
__device__ inline int wave_slot(int *n, bool take) {
  const int lane = threadIdx.x & 63;
  const unsigned long long m = __ballot(take);
  int base = 0;
  if (m && lane == __ffsll((long long)m) - 1) base = atomicAdd(n, __popcll(m));
  base = __shfl(base, __ffsll((long long)(m ? m : 1ull)) - 1, 64);
  return base + __popcll(m & (lane ? (~0ull >> (64 - lane)) : 0ull));
}

// Closed-interval overlap of two FP32 boxes (lo x, y, z, hi x, y, z) held in
// LDS at 8-byte aligned addresses: both boxes are read with three 8-byte
// loads each and the six compares are combined without branches (a
// short-circuit chain would wait for one pair of loads after another).
__device__ inline bool ov6f_lds(const float *A, const float *B) {
  const float2 a0 = *reinterpret_cast<const float2 *>(A), a1 = *reinterpret_cast<const float2 *>(A + 2),
               a2 = *reinterpret_cast<const float2 *>(A + 4);
  const float2 b0 = *reinterpret_cast<const float2 *>(B), b1 = *reinterpret_cast<const float2 *>(B + 2),
               b2 = *reinterpret_cast<const float2 *>(B + 4);
  // a0 = (lo x, lo y), a1 = (lo z, hi x), a2 = (hi y, hi z)
  return (a0.x <= b1.y) & (b0.x <= a1.y) & (a0.y <= b2.x) & (b0.y <= a2.x) & (a1.x <= b2.y) & (b1.x <= a2.y);
}

// Overlap of two patches' face-diagonal supports (9-DOP minus the box):
// A's unshifted, B's with the pair's shift already added.  The supports are
// rounded outward; the comparison in FP64 allows 1e-6 (1 + |x|) more, far
// above the roundings of the sums that formed them, so it never rejects a
// pair of patches that hold primitives with meeting boxes.
__device__ inline bool dop_meet(const float *A, const float *B) {
  bool ok = true;
#pragma unroll
  for (int j = 0; j < kDopDirs; ++j) {
    const double adn = A[2 * j], aup = A[2 * j + 1], bdn = B[2 * j], bup = B[2 * j + 1];
    ok &= (adn <= bup + 1e-6 * (1.0 + fabs(bup))) & (bdn <= aup + 1e-6 * (1.0 + fabs(aup)));
  }
  return ok;
}

// A vesicle pair's header is spread over the lanes of each wavefront, so
// the next pair's can be fetched while this pair is worked on, with one
// vector load per level, and read back with lane reads.  Level 1
// (pair_word): lane l < 6 holds 64-bit word l of the PairRec (lane 0: a, b;
// lanes 3-5: the image shift).  Level 2, 64-bit words (head_word): lanes 0-5
// A's box, 6-11 B's box (unshifted), 12-15 the patch-table offsets of A,
// A+1, B, B+1; 32-bit words (head_int): lanes 0-1 the vertex offsets of A
// and B, 2-3 their topology ids.  (Separate registers for the two widths:
// a 32-bit load merged into a 64-bit register would be waited for on the
// spot.)
__device__ inline uint64_t pair_word(const PairRec *pairs, int64_t p, int lane) {
  uint64_t v = 0;
  if (lane < 6) v = reinterpret_cast<const uint64_t *>(pairs + p)[lane];
  return v;
}

__device__ inline uint64_t head_word(const double *ves_box, const int64_t *ves_patch_off, uint64_t ab, int lane) {
  const int a = (int)(uint32_t)ab, b = (int)(uint32_t)(ab >> 32);
  uint64_t v = 0;
  if (lane < 12)
    v = (uint64_t)__double_as_longlong(ves_box[6 * (int64_t)(lane < 6 ? a : b) + lane % 6]);
  else if (lane < 16)
    v = (uint64_t)ves_patch_off[(lane < 14 ? a : b) + (lane & 1)];
  return v;
}

__device__ inline int head_int(const DevScene &S, uint64_t ab, int lane) {
  const int v = (lane & 1) ? (int)(uint32_t)(ab >> 32) : (int)(uint32_t)ab;
  int r = 0;
  if (lane < 2)
    r = S.vtx_off[v];
  else if (lane < 4)
    r = S.topo_id[v];
  return r;
}

__device__ inline uint64_t lane_word(uint64_t v, int l) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

// One workgroup per vesicle pair.  Each side's patch boxes that meet the
// other vesicle's box are staged in LDS as FP32 boxes rounded outward (a
// conservative filter: the primitive kernel applies the exact test later),
// with their face-diagonal supports; the surviving patch pairs are tested
// (boxes, then supports), and the work items are buffered in LDS and written
// with one atomic per flush.
// MAXP bounds the patches of any vesicle's topology (LDS is sized for it).
template <int MAXP>
__global__ __launch_bounds__(kPPThreads) void k_patch_pairs(DevScene S, DevTopo T, const PairRec *pairs,
                                                            const double *ves_box, const int64_t *ves_patch_off,
                                                            const double *patch_box, const float *patch_dop,
                                                            WorkRec *work, int64_t work_cap, Counters *cnt,
                                                            int64_t pairs_cap) {
  __shared__ alignas(8) float bA[MAXP][6];
  __shared__ alignas(8) float bB[MAXP][6];
  constexpr bool kDop = MAXP <= 512;  // larger meshes have no face-diagonal supports
  constexpr int kDopP = kDop ? MAXP : 1;
  __shared__ alignas(8) float dA[kDopP][kDopVals];
  __shared__ alignas(8) float dB[kDopP][kDopVals];
  __shared__ short iA[MAXP], iB[MAXP];
  __shared__ WorkRec buf[kPPBuf];
  __shared__ int nA, nB, nbuf;
  __shared__ unsigned long long base_sh;
  int64_t np = (int64_t)cnt->n_pairs;
  np = np < pairs_cap ? np : pairs_cap;
  if (threadIdx.x == 0) nbuf = 0;
  const int lane = threadIdx.x & 63;
  int64_t p = blockIdx.x;
  uint64_t prw = 0, hdw = 0;  // this pair's header (see pair_word, head_word, head_int)
  int hdi = 0;
  if (p < np) {
    prw = pair_word(pairs, p, lane);
    const uint64_t ab = lane_word(prw, 0);
    hdw = head_word(ves_box, ves_patch_off, ab, lane);
    hdi = head_int(S, ab, lane);
  }
  for (; p < np; p += gridDim.x) {
    double sh[3], boxA[6], boxB[6];
    for (int c = 0; c < 3; ++c) sh[c] = __longlong_as_double((long long)lane_word(prw, 3 + c));
    for (int c = 0; c < 6; ++c) boxA[c] = __longlong_as_double((long long)lane_word(hdw, c));
    for (int c = 0; c < 3; ++c) {
      boxB[c] = __longlong_as_double((long long)lane_word(hdw, 6 + c)) + sh[c];
      boxB[3 + c] = __longlong_as_double((long long)lane_word(hdw, 9 + c)) + sh[c];
    }
    const int64_t pa0 = (int64_t)lane_word(hdw, 12), pb0 = (int64_t)lane_word(hdw, 14);
    const int na = (int)((int64_t)lane_word(hdw, 13) - pa0), nb = (int)((int64_t)lane_word(hdw, 15) - pb0);
    const int vbA = __builtin_amdgcn_readlane(hdi, 0), vbB = __builtin_amdgcn_readlane(hdi, 1);
    const int ptA_v = T.patch_off[__builtin_amdgcn_readlane(hdi, 2)];
    const int ptB_v = T.patch_off[__builtin_amdgcn_readlane(hdi, 3)];
    // the next pair's record, in flight during this pair's patch loads
    const int64_t pn = p + gridDim.x;
    const uint64_t prw_n = pn < np ? pair_word(pairs, pn, lane) : 0;
    if (threadIdx.x == 0) { nA = 0; nB = 0; }
    __syncthreads();
    // compaction: a ballot per wavefront and one LDS atomic for its survivors.
    // Both vesicles' patches in one pass (A's, then B's), each thread loading
    // its patch's box and supports before any test: a pair waits for one
    // round of loads instead of four (A's boxes, A's supports, B's, B's).
    const double shd[kDopDirs] = {sh[0] + sh[1], sh[0] - sh[1], sh[0] + sh[2],
                                  sh[0] - sh[2], sh[1] + sh[2], sh[1] - sh[2]};
    for (int k0 = 0; k0 < na + nb; k0 += blockDim.x) {
      const int k = k0 + threadIdx.x;
      const bool inA = k < na, inB = !inA && k < na + nb;
      const int kk = inA ? k : k - na;
      double P[6];
      float D[kDopVals];
      bool keep = false;
      if (inA || inB) {
        const int64_t slot = inA ? pa0 + kk : pb0 + kk;
        for (int c = 0; c < 6; ++c) P[c] = patch_box[6 * slot + c];
        if (kDop)
          for (int j = 0; j < kDopVals; ++j) D[j] = patch_dop[kDopVals * slot + j];
        if (inB)
          for (int c = 0; c < 3; ++c) {
            P[c] += sh[c];
            P[3 + c] += sh[c];
          }
        const bool kA = ov6(P, boxB), kB = ov6(P, boxA);
        keep = inA ? kA : kB;
      }
      const int qa = wave_slot(&nA, keep && inA);
      const int qb = wave_slot(&nB, keep && inB);
      if (keep && inA) {
        for (int c = 0; c < 3; ++c) {
          bA[qa][c] = __double2float_rd(P[c]);
          bA[qa][3 + c] = __double2float_ru(P[3 + c]);
        }
        if (kDop)
          for (int j = 0; j < kDopVals; ++j) dA[qa][j] = D[j];
        iA[qa] = (short)kk;
      }
      if (keep && inB) {
        for (int c = 0; c < 3; ++c) {
          bB[qb][c] = __double2float_rd(P[c]);
          bB[qb][3 + c] = __double2float_ru(P[3 + c]);
        }
        // B's supports shifted by the image: (1,1,0).sh, (1,-1,0).sh, ...
        if (kDop)
          for (int j = 0; j < kDopDirs; ++j) {
            dB[qb][2 * j] = __double2float_rd((double)D[2 * j] + shd[j]);
            dB[qb][2 * j + 1] = __double2float_ru((double)D[2 * j + 1] + shd[j]);
          }
        iB[qb] = (short)kk;
      }
      // one pass covers both sides when 2 MAXP <= kPPThreads (the launch's
      // workgroup size): no loop back edge, across which the next pair's
      // loads in flight would be waited for before this pair's patch loads
      if (2 * MAXP <= kPPThreads) break;
    }
    // taken to scalars here, before the next pair's loads are issued: a later
    // use would wait for those too (loads complete in issue order)
    const int ptA = __builtin_amdgcn_readfirstlane(ptA_v), ptB = __builtin_amdgcn_readfirstlane(ptB_v);
    // the next pair's header, in flight during this pair's patch-pair tests
    uint64_t hdw_n = 0;
    int hdi_n = 0;
    if (pn < np) {
      const uint64_t ab = lane_word(prw_n, 0);
      hdw_n = head_word(ves_box, ves_patch_off, ab, lane);
      hdi_n = head_int(S, ab, lane);
    }
    __syncthreads();
    const int ma = nA, mb = nB;
    const int tot = ma * mb;
    for (int t0 = 0; t0 < tot; t0 += blockDim.x) {
      const int t = t0 + threadIdx.x;
      const int x = t < tot ? t / mb : 0, y = t < tot ? t - x * mb : 0;
      const bool hit = t < tot && ov6f_lds(bA[x], bB[y]) && (!kDop || dop_meet(dA[kDop ? x : 0], dB[kDop ? y : 0]));
      const int q = wave_slot(&nbuf, hit);
      {
        if (hit) {
          WorkRec w;
          w.p = (int)p;
          w.pa = ptA + iA[x];
          w.pb = ptB + iB[y];
          w.base_a = vbA;
          w.base_b = vbB;
          w.box_a = (int)(pa0 + iA[x]);
          w.box_b = (int)(pb0 + iB[y]);
          w.pad = 0;
          buf[q] = w;
        }
      }
      __syncthreads();
      if (nbuf > kPPBuf - kPPThreads) {  // flush
        if (threadIdx.x == 0) base_sh = atomicAdd(&cnt->n_work, (unsigned long long)nbuf);
        __syncthreads();
        for (int k = threadIdx.x; k < nbuf; k += blockDim.x)
          if ((int64_t)(base_sh + k) < work_cap) work[base_sh + k] = buf[k];
        __syncthreads();
        if (threadIdx.x == 0) nbuf = 0;
        __syncthreads();
      }
    }
    prw = prw_n;
    hdw = hdw_n;
    hdi = hdi_n;
    __syncthreads();
  }
  __syncthreads();
  if (nbuf > 0) {
    if (threadIdx.x == 0) base_sh = atomicAdd(&cnt->n_work, (unsigned long long)nbuf);
    __syncthreads();
    for (int k = threadIdx.x; k < nbuf; k += blockDim.x)
      if ((int64_t)(base_sh + k) < work_cap) work[base_sh + k] = buf[k];
  }
}

// --------------------------------------------------------------------------
// Per work item: one wavefront, both patches staged in LDS.
// 1. Staging.  The header and slot bytes of both patch blobs (BlobLayout),
//    the referenced vertex ids and the pair's image shift; then X0 and X1 of
//    every referenced vertex, kept in LDS in FP64, with each vertex's
//    space-time box rounded outward to FP32.  These are three dependent
//    rounds of global loads (work record; blobs; positions), so they are
//    software-pipelined across the work items of a wavefront: the record of
//    the item after next, the blobs of the next item and then its positions
//    are loaded into registers while the current item is swept, and only
//    written to LDS once the current item is finished.  A pair's items come
//    in the order of their first patch; an item with the pair and first
//    patch of the one before it loads and writes only its second patch.
//    The FP32 box of each whole patch comes from the box kernel's FP64 patch
//    box, rounded outward like the vertex boxes.
// 2. Per kind, build the left list (owned vertices, or owned edges; 64 at a
//    time) and the right list (triangles, or owned edges) of primitives whose
//    FP32 boxes meet the other patch's box; the FP32 boxes enclose the FP64
//    ones, so the filter keeps a superset.
// 3. All left x right pairs of the lists, 64 per round (two rounds' loads
//    issued together), FP32 box test; hits are buffered in LDS.
// 4. Buffered hits are processed 64 at a time with all lanes busy: the exact
//    FP64 box test (the candidate definition), then the screens: candidates
//    whose polynomial can have a root on [0,1] and whose closest-point test
//    can pass somewhere on [0,1] are listed in LDS and the rest are finished
//    here.
// 5. At the end of the item the listed candidates are queued for the
//    root-search kernel together with their FP64 geometry (structure of
//    arrays, so the root search reads them coalesced), with one atomic for
//    the item.  Nothing between the prefetch of the next item and its use
//    waits on a global load or on a returning atomic: the wait counter of
//    vector memory completes in order, so such a wait would also wait for
//    the prefetch.  The primitive ids come from the staged blob for the same
//    reason.
// --------------------------------------------------------------------------
constexpr int kHitBuf = 256;
constexpr int kQueueBuf = 256;  // candidates of one item listed for the root search

template <int TILE>
struct WaveLds {
  using Lay = BlobLayout<TILE>;
  static constexpr int kRef = TileCaps<TILE>::ref;
  static constexpr int kL = 64;  // the left-hand list is built 64 primitives at a time
  static constexpr int kR = TileCaps<TILE>::owne > TILE ? TileCaps<TILE>::owne : TILE;
  double pos[2][kRef][6];  // raw X0 (x, y, z), X1 (x, y, z) of the referenced vertices
  double sh[3];            // image shift of the pair
  float vbox[2][kRef][6];             // FP32 space-time box of each referenced vertex
  alignas(8) float lbox[kL][6];       // left-hand list (current chunk) of the current kind: FP32 boxes
  alignas(8) float rbox[kR][6];       // right-hand list
  uint8_t lk[kL];          // patch-local indices of the left-hand list
  uint8_t rk[kR];          // and of the right-hand list
  uint32_t hits[kHitBuf];  // kind << 16 | left << 8 | right (patch-local indices)
  uint32_t queued[kQueueBuf];  // hits of the current item that need the root search (same encoding)
  alignas(16) int blob[2][Lay::stage];  // header, slot and id arrays of the two patch blobs
};

// FP32 values at or below (above) x: the nearest float moved down (up) by
// 2^-22 of its magnitude, at least two units in its last place, plus 1e-30
// for values near zero.  Both maps are monotone in x, and cheaper than a
// conversion with a directed rounding.
__device__ inline float f32_down(double x) {
  const float f = (float)x;
  return f - (fabsf(f) * 2.384185791015625e-07f + 1e-30f);
}
__device__ inline float f32_up(double x) {
  const float f = (float)x;
  return f + (fabsf(f) * 2.384185791015625e-07f + 1e-30f);
}

// Overlap of two FP32 boxes in registers (branch-free).
__device__ inline bool ov6f(const float *A, const float *B) {
  return (A[0] <= B[3]) & (B[0] <= A[3]) & (A[1] <= B[4]) & (B[1] <= A[4]) & (A[2] <= B[5]) & (B[2] <= A[5]);
}

// FP64 box of a primitive (min - h + sh, max + h + sh), rounded outward to
// FP32, as the min / max of its vertices' FP32 boxes.  The map
// m -> f32_down(fl(fl(m - h) + sh)) is monotone, so the min over vertices
// of the rounded vertex bounds is the rounded bound of the min: the same box
// as rounding the primitive's FP64 box.
// nvert (1, 2 or 3) is wave-uniform.  All slot loads, then all box loads, are
// issued together (an edge repeats its second end as the third corner).
__device__ inline void prim_box32(const float (*vbox)[6], const uint8_t *slot, int nvert, float *out) {
  if (nvert == 1) {
#pragma unroll
    for (int c = 0; c < 6; ++c) out[c] = vbox[slot[0]][c];
    return;
  }
  const int s0 = slot[0], s1 = slot[1], s2 = slot[nvert - 1];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    out[c] = fminf(fminf(vbox[s0][c], vbox[s1][c]), vbox[s2][c]);
    out[3 + c] = fmaxf(fmaxf(vbox[s0][3 + c], vbox[s1][3 + c]), vbox[s2][3 + c]);
  }
}

template <int TILE>
__device__ inline const uint8_t *blob_bytes(const WaveLds<TILE> &W, int side, int off) {
  return reinterpret_cast<const uint8_t *>(&W.blob[side][off]);
}

// Queue the listed candidates of the current item (W.queued[0 .. nq), n_ee of
// them edge-edge) for
// the root search: keys with global primitive ids, and the FP64 geometry from
// LDS.  Vertex-triangle candidates fill the queue from its front, edge-edge
// ones from its back (so the root-search wavefronts are mostly of one kind,
// and those of edge-edge candidates skip the volume code); one atomic on the
// packed pair of counts for all of them.  All 64 lanes take part.
template <int TILE>
__device__ void flush_queued(WaveLds<TILE> &W, int p, Cand *hard, double *geo, int64_t hard_cap, Counters *cnt,
                             int nq, int n_ee) {
  using Lay = BlobLayout<TILE>;
  const int lane = threadIdx.x;
  const unsigned long long lt = lanemask_lt();
  unsigned long long b = 0;
  if (lane == 0)
    b = atomicAdd(&cnt->n_hard_vt_ee, ((unsigned long long)n_ee << 32) | (unsigned long long)(nq - n_ee));
  b = __shfl(b, 0, 64);
  unsigned long long b_vt = b & 0xffffffffull, b_ee = b >> 32;
  for (int r0 = 0; r0 < nq; r0 += 64) {
    const int k = r0 + lane;
    const uint32_t hv = k < nq ? W.queued[k] : 0u;
    const int kind = (int)((hv >> 16) & 3u), kl = (int)((hv >> 8) & 0xffu), kr = (int)(hv & 0xffu);
    const int sl = (kind == 1) ? 1 : 0, sr = 1 - sl;
    const bool ee = kind == 2;
    const unsigned long long m_ee = __ballot(k < nq && ee), m_vt = __ballot(k < nq && !ee);
    const unsigned long long r_ee = b_ee + __popcll(m_ee & lt), r_vt = b_vt + __popcll(m_vt & lt);
    b_ee += __popcll(m_ee);
    b_vt += __popcll(m_vt);
    if (k >= nq) break;
    // rank r from the back is slot hard_cap - 1 - r
    if ((int64_t)(ee ? r_ee : r_vt) >= hard_cap) continue;
    const unsigned long long slot = ee ? (unsigned long long)(hard_cap - 1) - r_ee : r_vt;
    int slots[4];
    if (ee) {
      const uint8_t *el = blob_bytes(W, sl, Lay::eslot), *er = blob_bytes(W, sr, Lay::eslot);
      slots[0] = el[2 * kl]; slots[1] = el[2 * kl + 1];
      slots[2] = er[2 * kr]; slots[3] = er[2 * kr + 1];
    } else {
      const uint8_t *vl = blob_bytes(W, sl, Lay::vslot), *tr = blob_bytes(W, sr, Lay::tslot);
      slots[0] = vl[kl];
      slots[1] = tr[3 * kr]; slots[2] = tr[3 * kr + 1]; slots[3] = tr[3 * kr + 2];
    }
    Cand c;
    c.pair = p;
    c.kind = kind;
    c.i = W.blob[sl][(ee ? Lay::pedge : Lay::pvtx) + kl];
    c.j = W.blob[sr][(ee ? Lay::pedge : Lay::ptri) + kr];
    hard[slot] = c;
    const int nfirst = ee ? 2 : 1;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int side = v >= nfirst ? sr : sl;
      const double *pp = W.pos[side][slots[v]];
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        geo[(3 * v + q) * hard_cap + slot] = pp[q] + (side ? W.sh[q] : 0.0);
        geo[(12 + 3 * v + q) * hard_cap + slot] = pp[3 + q] - pp[q];
      }
    }
  }
}

// Exact FP64 box test of a buffered hit and the polynomial screen; list the
// candidates that need a root search in W.queued (*nq of them; flushed
// early when the list could overflow).  All 64 lanes take part.  p is the
// pair of the current work item.
template <int N, int TILE>
__device__ void process_hits(WaveLds<TILE> &W, int p, double d, Cand *hard, double *geo, int64_t hard_cap,
                             Cand *list, int64_t list_cap, Counters *cnt, unsigned long long &nvt,
                             unsigned long long &nee, int nh, int &nq, int &nq_ee) {
  using Lay = BlobLayout<TILE>;
  const int lane = threadIdx.x;
  const double h = 0.5 * d;
  __syncthreads();
  for (int r0 = 0; r0 < nh; r0 += 64) {
    const int k = r0 + lane;
    bool is_cand = false, need = false;
    int kind = 0, kl = 0, kr = 0, sl = 0, sr = 1;
    uint32_t hv = 0;
    if (k < nh) {
      nm::Quad Q;
      hv = W.hits[k];
      kind = (int)((hv >> 16) & 3u);
      kl = (int)((hv >> 8) & 0xffu);
      kr = (int)(hv & 0xffu);
      sl = (kind == 1) ? 1 : 0;
      sr = 1 - sl;
      const bool ee = kind == 2;
      int slots[4];
      if (ee) {
        const uint8_t *el = blob_bytes(W, sl, Lay::eslot), *er = blob_bytes(W, sr, Lay::eslot);
        slots[0] = el[2 * kl]; slots[1] = el[2 * kl + 1];
        slots[2] = er[2 * kr]; slots[3] = er[2 * kr + 1];
      } else {
        const uint8_t *vl = blob_bytes(W, sl, Lay::vslot), *tr = blob_bytes(W, sr, Lay::tslot);
        slots[0] = vl[kl];
        slots[1] = tr[3 * kr]; slots[2] = tr[3 * kr + 1]; slots[3] = tr[3 * kr + 2];
      }
      // vertex k belongs to side sl for the first primitive, sr for the second
      const int nfirst = ee ? 2 : 1;
      Q.ee = ee;
      double lo[2][3], hi[2][3];
#pragma unroll
      for (int g = 0; g < 2; ++g)
#pragma unroll
        for (int q = 0; q < 3; ++q) { lo[g][q] = INFINITY; hi[g][q] = -INFINITY; }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const bool second = v >= nfirst;
        const int side = second ? sr : sl;
        const double *pp = W.pos[side][slots[v]];
        const double shx = side ? W.sh[0] : 0.0, shy = side ? W.sh[1] : 0.0, shz = side ? W.sh[2] : 0.0;
        Q.X0[v] = nm::mk(pp[0] + shx, pp[1] + shy, pp[2] + shz);
        Q.D[v] = nm::mk(pp[3] - pp[0], pp[4] - pp[1], pp[5] - pp[2]);
#pragma unroll
        for (int q = 0; q < 3; ++q) {
          const double mn = fmin(pp[q], pp[3 + q]), mx = fmax(pp[q], pp[3 + q]);
          if (second) { lo[1][q] = fmin(lo[1][q], mn); hi[1][q] = fmax(hi[1][q], mx); }
          else { lo[0][q] = fmin(lo[0][q], mn); hi[0][q] = fmax(hi[0][q], mx); }
        }
      }
      bool ov = true;
#pragma unroll
      for (int q = 0; q < 3; ++q) {
        const double s0 = sl ? W.sh[q] : 0.0, s1 = sr ? W.sh[q] : 0.0;
        const double l0 = (lo[0][q] - h) + s0, u0 = (hi[0][q] + h) + s0;
        const double l1 = (lo[1][q] - h) + s1, u1 = (hi[1][q] + h) + s1;
        ov = ov && l0 <= u1 && l1 <= u0;
      }
      if (ov) {
        is_cand = true;
        if (ee) ++nee; else ++nvt;
        need = nm::needs_root_search<N>(Q, d) && nm::may_be_inside(Q);
      }
    }
    // candidates for the root search: listed in LDS, queued at the end of the item
    const unsigned long long mh = __ballot(need);
    if (need) W.queued[nq + __popcll(mh & lanemask_lt())] = hv;
    nq += __popcll(mh);
    nq_ee += __popcll(__ballot(need && kind == 2));
    if (list) {
      // the optional candidate list (a diagnostic output): one atomic per round
      const unsigned long long mc = __ballot(is_cand);
      if (mc) {
        const int leader = __ffsll((long long)mc) - 1;
        unsigned long long b = 0;
        if (lane == leader) b = atomicAdd(&cnt->n_cand_list, (unsigned long long)__popcll(mc));
        b = __shfl(b, leader, 64);
        if (is_cand) {
          const unsigned long long slot = b + __popcll(mc & lanemask_lt());
          Cand c;
          c.pair = p;
          c.kind = kind;
          const bool ee = kind == 2;
          c.i = W.blob[sl][(ee ? Lay::pedge : Lay::pvtx) + kl];
          c.j = W.blob[sr][(ee ? Lay::pedge : Lay::ptri) + kr];
          if ((int64_t)slot < list_cap) list[slot] = c;
        }
      }
    }
    if (nq > kQueueBuf - 64) {  // rare: a long list is queued before the item ends
      __syncthreads();
      flush_queued<TILE>(W, p, hard, geo, hard_cap, cnt, nq, nq_ee);
      nq = 0;
      nq_ee = 0;
      __syncthreads();
    }
  }
  __syncthreads();
}

// Registers of a work item in flight: its record (lanes 0-7 hold the eight
// ints of WorkRec), the pair's image shift (lanes 0-2), the FP64 boxes of both
// patches (lanes 0-11), the staged part of both blobs (header, slots and ids:
// two int4 per lane), the referenced vertex ids and, once those have arrived,
// the positions of the referenced vertices.
template <int TILE>
struct Prefetch {
  using Lay = BlobLayout<TILE>;
  static_assert(Lay::stage / 4 <= 128 && Lay::ref <= 64, "two int4 of each blob and one vertex per lane");
  int4 blob[2][2];
  int ref[2];
  double sh;
  double pbox;  // lanes 0-11: the FP64 box of patch lane / 6, component lane % 6
  double pos[2][6];
};

// Work items are handed out in chunks of kChunk consecutive items: wavefront b
// starts with chunk b, and claims each further chunk from a device counter as
// it enters a chunk, kChunk items before it needs it (so the atomic's latency
// is hidden and there is one atomic per kChunk items).  Items differ widely in
// cost; fixed strides left the last 30 % of the kernel with few wavefronts.
constexpr int kChunk = 8;

struct ItemSeq {
  int end;      // end of the chunk of the last item handed out
  int pending;  // lane 0: first item of the chunk claimed next (read when needed)
};

__device__ inline int claim_chunk(Counters *cnt, int64_t first_dynamic, int lane) {
  unsigned long long t = 0;
  if (lane == 0) t = first_dynamic + (unsigned long long)kChunk * atomicAdd(&cnt->work_claimed, 1ull);
  return (int)(t < 0x7fffffffull ? t : 0x7fffffffull);
}

// The item after `last` in this wavefront's sequence.
__device__ inline int next_item(int last, ItemSeq &Q, Counters *cnt, int64_t first_dynamic, int lane) {
  if (last + 1 < Q.end) return last + 1;
  const int start = __builtin_amdgcn_readfirstlane(Q.pending);
  Q.pending = claim_chunk(cnt, first_dynamic, lane);
  Q.end = start + kChunk;
  return start;
}

__device__ inline int load_workrec(const WorkRec *work, int64_t w, int64_t nw, int lane) {
  return (w < nw && lane < 8) ? reinterpret_cast<const int *>(work + w)[lane] : 0;
}

// Blobs, referenced ids, patch boxes and shift of a work item whose record is
// in wr.  With keep0 (wave-uniform: the item has the same pair and first patch
// as the one before it) the first patch's registers are left as they are.
template <int TILE>
__device__ inline void load_blobs(Prefetch<TILE> &F, const DevTopo &T, const PairRec *pairs, const double *patch_box,
                                  int wr, int lane, bool keep0) {
  using Lay = BlobLayout<TILE>;
  const int p = __builtin_amdgcn_readlane(wr, 0);
  const int P[2] = {__builtin_amdgcn_readlane(wr, 1), __builtin_amdgcn_readlane(wr, 2)};
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    if (side == 0 && keep0) continue;
    const int *gb = T.blob + (int64_t)P[side] * Lay::stride;
#pragma unroll
    for (int h = 0; h < 2; ++h)
      F.blob[side][h] =
          64 * h + lane < Lay::stage / 4 ? reinterpret_cast<const int4 *>(gb)[64 * h + lane] : int4{0, 0, 0, 0};
    // unused entries of the referenced list are 0: a valid vertex of the vesicle
    F.ref[side] = lane < Lay::ref ? gb[Lay::pref + lane] : 0;
  }
  F.sh = lane < 3 ? pairs[p].sh[lane] : 0.0;
  const int box[2] = {__builtin_amdgcn_readlane(wr, 5), __builtin_amdgcn_readlane(wr, 6)};
  if (lane < 12 && !(keep0 && lane < 6)) F.pbox = patch_box[6 * (int64_t)box[lane >= 6] + lane % 6];
}

// Positions of the referenced vertices (every lane below the list capacity
// loads one vertex; lanes past the patch's count load vertex 0 of the vesicle).
template <int TILE>
__device__ inline void load_positions(Prefetch<TILE> &F, const DevScene &S, int wr, int lane, bool keep0) {
  using Lay = BlobLayout<TILE>;
  const int base[2] = {__builtin_amdgcn_readlane(wr, 3), __builtin_amdgcn_readlane(wr, 4)};
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    if (side == 0 && keep0) continue;
    if (lane < Lay::ref) {
      const int64_t g = base[side] + F.ref[side];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        F.pos[side][c] = S.x0[c * (int64_t)S.n_vtx + g];
        F.pos[side][3 + c] = S.x1[c * (int64_t)S.n_vtx + g];
      }
    }
  }
}

template <int N, int TILE>
__global__ __launch_bounds__(64) void k_prim_cand(DevScene S, DevTopo T, const PairRec *pairs, const WorkRec *work,
                                                  int64_t work_cap, const double *patch_box, double d, Cand *hard, double *geo,
                                                  int64_t hard_cap, Cand *list, int64_t list_cap, Counters *cnt) {
  using Lay = BlobLayout<TILE>;
  __shared__ WaveLds<TILE> W;
  const int lane = threadIdx.x;
  const double h = 0.5 * d;
  int64_t nw = (int64_t)cnt->n_work;
  nw = nw < work_cap ? nw : work_cap;
  unsigned long long nvt = 0, nee = 0, ntests = 0, npre = 0;
  // this wavefront's items: its own first chunk, then chunks claimed in turn
  const int64_t first_dynamic = (int64_t)gridDim.x * kChunk;
  ItemSeq Q;
  Q.end = (int)(blockIdx.x * kChunk + kChunk);
  Q.pending = claim_chunk(cnt, first_dynamic, lane);
  int w = (int)(blockIdx.x * kChunk);
  int w_next = next_item(w, Q, cnt, first_dynamic, lane);
  // pipeline prologue: the first item completely, the record of the second
  Prefetch<TILE> F;
  int wr_cur = load_workrec(work, w, nw, lane);
  int wr_next = load_workrec(work, w_next, nw, lane);
  if (w < nw) {
    load_blobs<TILE>(F, T, pairs, patch_box, wr_cur, lane, false);
    load_positions<TILE>(F, S, wr_cur, lane, false);
  }
  // the current item has the pair and first patch of the previous one: that
  // patch's blob, positions and vertex boxes are still in LDS (consecutive
  // items of a pair come in the order of the first patch)
  bool same0 = false;
  while (w < nw) {
    // the current item: registers -> LDS
    const int p = __builtin_amdgcn_readlane(wr_cur, 0);
    const int P[2] = {__builtin_amdgcn_readlane(wr_cur, 1), __builtin_amdgcn_readlane(wr_cur, 2)};
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      if (side == 0 && same0) continue;
#pragma unroll
      for (int h = 0; h < 2; ++h)
        if (64 * h + lane < Lay::stage / 4) reinterpret_cast<int4 *>(&W.blob[side][0])[64 * h + lane] = F.blob[side][h];
      if (lane < Lay::ref)
#pragma unroll
        for (int c = 0; c < 6; ++c) W.pos[side][lane][c] = F.pos[side][c];
    }
    if (lane < 3) W.sh[lane] = F.sh;
    __syncthreads();
    // FP32 boxes of the referenced vertices, rounded outward, into LDS
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      if (side == 0 && same0) continue;
      const int nref = W.blob[side][Lay::hdr + 0];
      if (lane < nref) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double a = F.pos[side][c], b = F.pos[side][3 + c];
          const double sc = side ? W.sh[c] : 0.0;
          W.vbox[side][lane][c] = f32_down((fmin(a, b) - h) + sc);
          W.vbox[side][lane][3 + c] = f32_up((fmax(a, b) + h) + sc);
        }
      }
    }
    // the two patch boxes in FP32 (wave-uniform).  The FP64 patch box is
    // fl(m - h) with m the exact minimum (maximum) over the patch's vertices,
    // and x -> f32_down(fl(fl(x - h) + s)) is monotone, so this equals the
    // union of the vertex boxes above.
    float pb[2][6];
    {
      float v = 0.0f;
      if (lane < 12) {
        const int c = lane % 6;
        const double x = F.pbox + (lane >= 6 ? W.sh[c % 3] : 0.0);
        v = c < 3 ? f32_down(x) : f32_up(x);
      }
#pragma unroll
      for (int side = 0; side < 2; ++side)
#pragma unroll
        for (int c = 0; c < 6; ++c)
          pb[side][c] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 6 * side + c));
    }
    // the next item's blobs and the record of the one after it (the loads
    // complete while this item is swept)
    const bool more = w_next < nw;
    const bool same0_next =
        more && __builtin_amdgcn_readlane(wr_next, 0) == p && __builtin_amdgcn_readlane(wr_next, 1) == P[0];
    if (more) load_blobs<TILE>(F, T, pairs, patch_box, wr_next, lane, same0_next);
    const int w_after = next_item(w_next, Q, cnt, first_dynamic, lane);
    const int wr_after = load_workrec(work, w_after, nw, lane);
    __syncthreads();
    int nh = 0;  // buffered hits (wave-uniform)
    int nq = 0, nq_ee = 0;  // listed candidates of this item, and its edge-edge ones (wave-uniform)
    for (int kind = 0; kind < 3; ++kind) {
      if (kind == 1 && more) load_positions<TILE>(F, S, wr_next, lane, same0_next);
      const int sl = (kind == 1) ? 1 : 0, sr = 1 - sl;
      const int lcount = kind == 2 ? W.blob[sl][Lay::hdr + 3] : W.blob[sl][Lay::hdr + 1];
      const int rcount = kind == 2 ? W.blob[sr][Lay::hdr + 3] : W.blob[sr][Lay::hdr + 2];
      const uint8_t *lslot = blob_bytes(W, sl, kind == 2 ? Lay::eslot : Lay::vslot);
      const uint8_t *rslot = blob_bytes(W, sr, kind == 2 ? Lay::eslot : Lay::tslot);
      const int lnv = kind == 2 ? 2 : 1;
      const int rnv = kind == 2 ? 2 : 3;
      // compact the primitives whose box meets the other patch's box (ballot +
      // prefix count): the right-hand list whole, the left-hand list 64 at a time
      int nr = 0;
      for (int k0 = 0; k0 < rcount; k0 += 64) {
        const int k = k0 + lane;
        float bx[6];
        bool keep = false;
        if (k < rcount) {
          prim_box32(W.vbox[sr], rslot + rnv * k, rnv, bx);
          keep = ov6f(bx, pb[sl]);
        }
        const unsigned long long m = __ballot(keep);
        if (keep) {
          const int q = nr + __popcll(m & lanemask_lt());
#pragma unroll
          for (int c = 0; c < 6; ++c) W.rbox[q][c] = bx[c];
          W.rk[q] = (uint8_t)k;
        }
        nr += __popcll(m);
      }
      // the sweep's lanes step through t = x * nr + y by 64 = q64 * nr + r64
      const int q64 = nr ? 64 / nr : 0, r64 = 64 - q64 * nr;
      const int x_lane = nr ? threadIdx.x / nr : 0, y_lane = threadIdx.x - x_lane * nr;
      for (int l0 = 0; l0 < (nr ? lcount : 0); l0 += 64) {
        const int k = l0 + lane;
        float bx[6];
        bool keep = false;
        if (k < lcount) {
          prim_box32(W.vbox[sl], lslot + lnv * k, lnv, bx);
          keep = ov6f(bx, pb[sr]);
        }
        const unsigned long long m = __ballot(keep);
        if (keep) {
          const int q = __popcll(m & lanemask_lt());
#pragma unroll
          for (int c = 0; c < 6; ++c) W.lbox[q][c] = bx[c];
          W.lk[q] = (uint8_t)k;
        }
        const int nl = __popcll(m);
        __syncthreads();
        // all left x right pairs, 64 per round: lane tests pair (x, y) of
        // t = x * nr + y, and (x, y) advances by 64 each round without a
        // division (t < nl * nr exactly when x < nl)
        const int tot = nl * nr;
        ntests += (unsigned long long)tot;
        int xr = x_lane, yr = y_lane;
        // two rounds per iteration, every load of both issued before either
        // ballot (lanes past the end test pair 0 and discard it)
        for (int t0 = 0; t0 < tot; t0 += 128) {
          int xn = xr + q64, yn = yr + r64;
          if (yn >= nr) { yn -= nr; ++xn; }
          const bool va = xr < nl, vb = xn < nl;
          const int xa = va ? xr : 0, ya = va ? yr : 0, xb = vb ? xn : 0, yb = vb ? yn : 0;
          xr = xn + q64;
          yr = yn + r64;
          if (yr >= nr) { yr -= nr; ++xr; }
          const bool ha = va & ov6f_lds(W.lbox[xa], W.rbox[ya]);
          const bool hb = vb & ov6f_lds(W.lbox[xb], W.rbox[yb]);
          const uint32_t ra = ((uint32_t)kind << 16) | ((uint32_t)W.lk[xa] << 8) | (uint32_t)W.rk[ya];
          const uint32_t rb = ((uint32_t)kind << 16) | ((uint32_t)W.lk[xb] << 8) | (uint32_t)W.rk[yb];
          const unsigned long long ma = __ballot(ha), mb = __ballot(hb);
          if (ha) W.hits[nh + __popcll(ma & lanemask_lt())] = ra;
          nh += __popcll(ma);
          if (hb) W.hits[nh + __popcll(mb & lanemask_lt())] = rb;
          nh += __popcll(mb);
          if (nh > kHitBuf - 128) {
            process_hits<N, TILE>(W, p, d, hard, geo, hard_cap, list, list_cap, cnt, nvt, nee, nh, nq, nq_ee);
            npre += (unsigned long long)nh;
            nh = 0;
          }
        }
        __syncthreads();
      }
    }
    // the hits refer to this item's LDS data: finish them before the next item
    if (nh) {
      process_hits<N, TILE>(W, p, d, hard, geo, hard_cap, list, list_cap, cnt, nvt, nee, nh, nq, nq_ee);
      npre += (unsigned long long)nh;
    }
    if (nq) flush_queued<TILE>(W, p, hard, geo, hard_cap, cnt, nq, nq_ee);
    w = w_next;
    w_next = w_after;
    wr_cur = wr_next;
    wr_next = wr_after;
    same0 = same0_next;
  }
  for (int off = 32; off > 0; off >>= 1) {
    nvt += __shfl_xor(nvt, off, 64);
    nee += __shfl_xor(nee, off, 64);
  }
  if (lane == 0) {
    if (nvt) atomicAdd(&cnt->n_cand_vt, nvt);
    if (nee) atomicAdd(&cnt->n_cand_ee, nee);
    if (ntests) atomicAdd(&cnt->n_tests, ntests);
    if (npre) atomicAdd(&cnt->n_pre, npre);
  }
}

}  // namespace

void launch_patch_pairs(const DevScene &S, const DevTopo &T, const PairRec *pairs, int64_t pairs_cap,
                        const double *ves_box, const int64_t *ves_patch_off, const double *patch_box,
                        const float *patch_dop, WorkRec *work, int64_t work_cap, int max_patches, Counters *cnt,
                        hipStream_t st) {
  // grids measured on the 1440-vesicle scene (order-32 meshes): 1024
  // workgroups, each taking several pairs into its work-item buffer before a
  // flush, 0.045 ms; 2048: 0.054; 4096: 0.067; 512: 0.062
  if (max_patches <= 128)
    k_patch_pairs<128><<<1024, kPPThreads, 0, st>>>(S, T, pairs, ves_box, ves_patch_off, patch_box, patch_dop, work,
                                                    work_cap, cnt, pairs_cap);
  else if (max_patches <= 512)
    k_patch_pairs<512><<<2048, kPPThreads, 0, st>>>(S, T, pairs, ves_box, ves_patch_off, patch_box, patch_dop, work,
                                                    work_cap, cnt, pairs_cap);
  else
    k_patch_pairs<kMaxPatchesPerVes><<<2048, kPPThreads, 0, st>>>(S, T, pairs, ves_box, ves_patch_off, patch_box,
                                                                  patch_dop, work, work_cap, cnt, pairs_cap);
}

template <int TILE>
static void launch_tile(int blocks, const DevScene &S, const DevTopo &T, const PairRec *pairs, const WorkRec *work,
                        int64_t work_cap, const double *patch_box, double d, Cand *hard, double *geo, int64_t hard_cap, Cand *list,
                        int64_t list_cap, Counters *cnt, hipStream_t st) {
  if (d == 0.0)
    k_prim_cand<3, TILE><<<blocks, 64, 0, st>>>(S, T, pairs, work, work_cap, patch_box, d, hard, geo, hard_cap, list, list_cap,
                                              cnt);
  else
    k_prim_cand<6, TILE><<<blocks, 64, 0, st>>>(S, T, pairs, work, work_cap, patch_box, d, hard, geo, hard_cap, list, list_cap,
                                              cnt);
}

void launch_prim_cand(int tile, int blocks, const DevScene &S, const DevTopo &T, const PairRec *pairs,
                      const WorkRec *work, int64_t work_cap, const double *patch_box, double d, Cand *hard,
                      double *hard_geo,
                      int64_t hard_cap, Cand *list, int64_t list_cap, Counters *cnt, hipStream_t st) {
  if (tile <= 16)
    launch_tile<16>(blocks, S, T, pairs, work, work_cap, patch_box, d, hard, hard_geo, hard_cap, list, list_cap, cnt, st);
  else if (tile <= 32)
    launch_tile<32>(blocks, S, T, pairs, work, work_cap, patch_box, d, hard, hard_geo, hard_cap, list, list_cap, cnt, st);
  else
    launch_tile<64>(blocks, S, T, pairs, work, work_cap, patch_box, d, hard, hard_geo, hard_cap, list, list_cap, cnt, st);
}

}  // namespace stiv
