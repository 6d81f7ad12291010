// K3 + K4: narrow phase (Eq. 3.1) and contact volume with its gradient
// (Eq. 3.2, App. A), FP64, one thread per queued candidate.  The candidates
// arrive here only when the screen in the primitive kernel could not exclude
// a root on [0,1] (see k_prim.hip).
//
// Trajectories are linear: P(s) = X0 + s D with D = X1 - X0 and s = t/dt in
// [0,1].  For a triangle (a,b,c) and vertex p, e1 = Pb - Pa, e2 = Pc - Pa,
// w = Pp - Pa, n = e1 x e2; g = w.n is cubic in s, q = |n|^2 quartic, and the
// vertex is within d of the triangle's plane where F = g^2 - d^2 q <= 0.  For
// edges (a,b), (c,e) the normal is (Pb - Pa) x (Pe - Pc) and w = Pc - Pa.
// With d = 0 the condition is g = 0.
//
// The earliest valid root is found by Bernstein-basis subdivision: on each
// dyadic interval the polynomial is re-expanded in the Bernstein basis; a
// block of one sign proves there is no root, a single sign change proves
// exactly one (variation diminishing), which is then bracketed by
// bisection to a width of 2^-50.  Intervals are visited depth-first, left
// to right, without a stack (the dyadic index itself encodes the traversal),
// so the first root whose closest point lies inside the triangle (resp. both
// segments) is the earliest contact.  A vertex already within d and inside
// at s = 0 is in contact at s = 0.
//
// For a vertex-triangle contact at s*:  V = (dt - tau) sqrt(eps^2 +
// (U.nhat)^2) |t| = 0.5 dt (1 - s) R with R = sqrt(eps^2 q + (U.n)^2) and
// U = D_p / dt; the gradient w.r.t. X1 (X0 fixed) adds the explicit
// dependence through P(s*) and U to dV/ds * ds/dX1, with ds/dX1 from the
// implicit function theorem on F(s*, X1) = 0.
//
// Learned bracket (optional): a small perceptron (mlp_tile.h) predicts the
// contact time of each queued candidate from its shape (the other three
// vertices relative to the first vertex of the triangle, resp. of the first
// edge, at both ends of the step, over the mean edge length at t_n), on the
// matrix cores with its activations in registers.  When [0, 1] is undecided
// the search certifies [0, lo) root-free with one Bernstein test and then
// traverses [lo, hi] and [hi, 1] instead of the halves of [0, 1], and the
// prediction starts the refinement of the root it lies in (search_in in
// narrow_math.h); the contacts found are the same as without it.
#include "mlp_tile.h"
#include "narrow_math.h"

namespace stiv {

namespace {

using namespace nm;

__device__ inline unsigned long long lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}


// Geometry of queued candidate i (written by the primitive kernel, structure
// of arrays [24][cap]): X0 of vertices 0..3 (image shift applied), then
// D = X1 - X0; order (p, a, b, c) for vertex-triangle, (a, b, c, e) for
// edge-edge.  Coalesced: consecutive threads read consecutive candidates.
__device__ inline void load_geo(const double *geo, int64_t cap, int64_t i, bool ee, Quad &Q) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    Q.X0[v] = mk(geo[(3 * v + 0) * cap + i], geo[(3 * v + 1) * cap + i], geo[(3 * v + 2) * cap + i]);
    Q.D[v] = mk(geo[(12 + 3 * v + 0) * cap + i], geo[(12 + 3 * v + 1) * cap + i], geo[(12 + 3 * v + 2) * cap + i]);
  }
  Q.ee = ee;
}

__device__ inline float len3f(const d3 &v) {
  const float x = (float)v.x, y = (float)v.y, z = (float)v.z;
  return sqrtf(x * x + y * y + z * z);
}

// Features of the learned bracket from the candidate's positions (selects,
// not indices, pick the vertices so that Q stays in registers).  Differences
// are taken in FP64 and the rest in FP32 (the network reads bf16).
__device__ inline void bracket_features(const Quad &Q, float out[mlp::kIn]) {
  const bool ee = Q.ee;
  float ell;
  if (ee) {
    ell = 0.5f * (len3f(Q.X0[1] - Q.X0[0]) + len3f(Q.X0[3] - Q.X0[2]));
  } else {
    ell = (len3f(Q.X0[2] - Q.X0[1]) + len3f(Q.X0[3] - Q.X0[1]) + len3f(Q.X0[3] - Q.X0[2])) * (1.0f / 3.0f);
  }
  const float inv = ell > 0.0f ? 1.0f / ell : 1.0f;
  const d3 A0 = ee ? Q.X0[0] : Q.X0[1], AD = ee ? Q.D[0] : Q.D[1];
  const d3 P0[3] = {ee ? Q.X0[1] : Q.X0[2], ee ? Q.X0[2] : Q.X0[3], ee ? Q.X0[3] : Q.X0[0]};
  const d3 PD[3] = {ee ? Q.D[1] : Q.D[2], ee ? Q.D[2] : Q.D[3], ee ? Q.D[3] : Q.D[0]};
  const d3 A1 = A0 + AD;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const d3 a = P0[r] - A0;
    const d3 b = (P0[r] + PD[r]) - A1;
    out[3 * r + 0] = (float)a.x * inv;
    out[3 * r + 1] = (float)a.y * inv;
    out[3 * r + 2] = (float)a.z * inv;
    out[9 + 3 * r + 0] = (float)b.x * inv;
    out[9 + 3 * r + 1] = (float)b.y * inv;
    out[9 + 3 * r + 2] = (float)b.z * inv;
  }
}

// Adds each lane's 1 to cnt[key] with one atomic per distinct key of the
// wavefront (lanes with key < 0 take no part): the contacts per vesicle pair
// that the aggregation buckets by.
__device__ inline void wave_count(int32_t *ctr, int key) {
  const int lane = threadIdx.x & 63;
  unsigned long long todo = __ballot(key >= 0);
  while (todo) {
    const int leader = __ffsll((long long)todo) - 1;
    const int k0 = __shfl(key, leader, 64);
    const unsigned long long grp = __ballot(key == k0) & todo;
    if (lane == leader) atomicAdd(&ctr[k0], __popcll(grp));
    todo &= ~grp;
  }
}

// Slot of queue index i (vertex-triangle candidates first, then edge-edge
// ones, which fill the queue from its back).
__device__ inline int64_t queue_slot(int64_t i, int64_t n_vt, int64_t cap) { return i < n_vt ? i : cap - 1 - (i - n_vt); }

struct BracketLds {
  mlp::Weights W;
  alignas(16) unsigned short x[256][mlp::kXS];
};

// Root search on the queued candidates, then volume and gradient on contact.
// LEARNED: the bracket of every candidate is predicted first (all 256
// candidates of the workgroup through the perceptron on the matrix cores).
template <int N, bool LEARNED>
__global__ __launch_bounds__(256) void k_narrow(const Cand *hard, const double *geo, int64_t hard_cap, double d,
                                                double eps,
                                                double dt, Cand *ct, double *ct_s, double *ct_vol, double *ct_grad,
                                                int64_t ct_cap, int32_t *pair_cnt, const void *mlp_packed,
                                                float kwidth, Counters *cnt) {
  // the queue: vertex-triangle candidates at its front, edge-edge ones at
  // its back; index i < n_vt is slot i, the others count from the back
  const unsigned long long vt_ee = cnt->n_hard_vt_ee;
  int64_t n_vt = (int64_t)(vt_ee & 0xffffffffull), n_ee = (int64_t)(vt_ee >> 32);
  n_vt = n_vt < hard_cap ? n_vt : hard_cap;
  n_ee = n_ee < hard_cap - n_vt ? n_ee : hard_cap - n_vt;
  const int64_t nc = n_vt + n_ee;
  int within = 0, deg = 0, exh = 0, cert = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  extern __shared__ char dyn_lds[];
  BracketLds &L = *reinterpret_cast<BracketLds *>(dyn_lds);
  if (LEARNED) {
    if ((int64_t)blockIdx.x * blockDim.x >= nc) return;  // whole workgroup idle: uniform exit
    mlp::load_packed(L.W, reinterpret_cast<const mlp::Weights *>(mlp_packed));
    __syncthreads();  // the only workgroup barrier: after it each wavefront uses its own LDS rows
  }
  // Plain search: the next candidate's record and geometry are loaded while
  // the current one is searched (the loop's only global loads; in-order
  // completion would otherwise expose their latency every iteration).  The
  // learned search has no registers to spare for that and loads each
  // candidate once, at the start of its iteration.
  Cand cn;
  Quad Qn;
  cn.pair = cn.kind = cn.i = cn.j = 0;
  if (!LEARNED) {
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i0 < nc) {
      const int64_t q = queue_slot(i0, n_vt, hard_cap);
      cn = hard[q];
      load_geo(geo, hard_cap, q, cn.kind == 2, Qn);
    }
  }
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nc; base += stride) {
    const int64_t i = base + threadIdx.x;
    int hit = 0;
    double s = 0.0, V = 0.0, g[12];
    if (LEARNED && i < nc) {
      const int64_t q = queue_slot(i, n_vt, hard_cap);
      cn = hard[q];
      load_geo(geo, hard_cap, q, cn.kind == 2, Qn);
    }
    const Cand c = cn;
    const Quad Q = Qn;
    for (int k = 0; k < 12; ++k) g[k] = 0.0;
    if (!LEARNED && i + stride < nc) {
      const int64_t q = queue_slot(i + stride, n_vt, hard_cap);
      cn = hard[q];
      load_geo(geo, hard_cap, q, cn.kind == 2, Qn);
    }
    if (LEARNED) {
      {
        float ft[mlp::kIn];
        if (i < nc) {
          bracket_features(Q, ft);
        } else {
#pragma unroll
          for (int k = 0; k < mlp::kIn; ++k) ft[k] = 0.0f;
        }
        // the row as eight 8-byte stores (columns kIn .. kInP - 1 are zero)
#pragma unroll
        for (int q = 0; q < mlp::kInP / 4; ++q) {
          mlp::bf16x4 v;
#pragma unroll
          for (int j = 0; j < 4; ++j) v[j] = (short)(4 * q + j < mlp::kIn ? mlp::f2bf(ft[4 * q + j]) : 0);
          *reinterpret_cast<mlp::bf16x4 *>(&L.x[threadIdx.x][4 * q]) = v;
        }
      }
      mlp::wave_lds_sync();
      // the wavefront's 64 samples, 16 at a time; the outputs of sample
      // 16 q + c arrive in lane c and go to the lane that owns the sample
      const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
      float o_mu = 0.0f, o_sd = 0.0f;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const mlp::f32x4 o = mlp::forward_t16(L.W, &L.x[64 * wave + 16 * q][0]);
        const float a = __shfl(o[0], lane & 15, 64), b = __shfl(o[1], lane & 15, 64);
        if ((lane >> 4) == q) {
          o_mu = a;
          o_sd = b;
        }
      }
      if (i < nc) {
        const float mu = mlp::head_mu(o_mu), sd = mlp::head_sd(o_sd);
        double lo = (double)mu - (double)kwidth * (double)sd, hi = (double)mu + (double)kwidth * (double)sd;
        lo = lo < 0.0 ? 0.0 : lo;
        hi = hi > 1.0 ? 1.0 : hi;
        int certified = 0;
        hit = earliest_bracket<N>(Q, d, lo, hi, (double)mu, &s, &within, &deg, &exh, &certified);
        cert += certified;
      }
      mlp::wave_lds_sync();
    } else if (i < nc) {
      hit = earliest<N>(Q, d, &s, &within, &deg, &exh);
    }
    if (hit && !Q.ee) volume_grad(Q, s, d, eps, dt, s == 0.0, &V, g);
    const unsigned long long m = __ballot(hit != 0);
    const int nh = __popcll(m);
    const int leader = m ? __ffsll((long long)m) - 1 : 0;
    const int nee_w = __popcll(__ballot(hit != 0 && c.kind == 2));
    unsigned long long slot0 = 0;
    if ((int)(threadIdx.x & 63) == leader && nh) {
      slot0 = atomicAdd(&cnt->n_ct, (unsigned long long)nh);
      if (nee_w) atomicAdd(&cnt->n_ct_ee, (unsigned long long)nee_w);
      if (nh - nee_w) atomicAdd(&cnt->n_ct_vt, (unsigned long long)(nh - nee_w));
    }
    slot0 = __shfl(slot0, leader, 64);
    const unsigned long long slot = slot0 + __popcll(m & lanemask_lt());
    // the stored contacts, counted per vesicle pair
    wave_count(pair_cnt, hit && (int64_t)slot < ct_cap ? c.pair : -1);
    if (hit) {
      if ((int64_t)slot < ct_cap) {
        ct[slot] = c;
        ct_s[slot] = s;
        ct_vol[slot] = V;
        for (int k = 0; k < 12; ++k) ct_grad[12 * slot + k] = g[k];
      }
    }
  }
  if (within) atomicAdd(&cnt->within_d, (unsigned long long)within);
  if (deg) atomicAdd(&cnt->degenerate, (unsigned long long)deg);
  if (exh) atomicAdd(&cnt->search_exhausted, (unsigned long long)exh);
  if (LEARNED && cert) atomicAdd(&cnt->n_bracket_ok, (unsigned long long)cert);
}

}  // namespace

static int grid_for(int64_t n, int max_blocks) {
  int64_t g = (n + 255) / 256;
  if (g > max_blocks) g = max_blocks;
  if (g < 1) g = 1;
  return (int)g;
}

void launch_narrow(int blocks, const DevScene &S, const DevTopo &T, const PairRec *pairs, const Cand *hard,
                   const double *hard_geo, int64_t hard_cap, double d, double eps, double dt, Cand *ct, double *ct_s,
                   double *ct_vol, double *ct_grad, int64_t ct_cap, int32_t *pair_cnt, const void *mlp_packed,
                   float kwidth, Counters *cnt, hipStream_t st) {
  (void)S; (void)T; (void)pairs;
  const int g = grid_for(hard_cap, blocks);
  const size_t lds = sizeof(BracketLds);
  if (mlp_packed) {
    if (d == 0.0)
      k_narrow<3, true><<<g, 256, lds, st>>>(hard, hard_geo, hard_cap, d, eps, dt, ct, ct_s, ct_vol, ct_grad, ct_cap,
                                            pair_cnt, mlp_packed, kwidth, cnt);
    else
      k_narrow<6, true><<<g, 256, lds, st>>>(hard, hard_geo, hard_cap, d, eps, dt, ct, ct_s, ct_vol, ct_grad, ct_cap,
                                            pair_cnt, mlp_packed, kwidth, cnt);
  } else {
    if (d == 0.0)
      k_narrow<3, false><<<g, 256, 0, st>>>(hard, hard_geo, hard_cap, d, eps, dt, ct, ct_s, ct_vol, ct_grad, ct_cap,
                                           pair_cnt, nullptr, 0.0f, cnt);
    else
      k_narrow<6, false><<<g, 256, 0, st>>>(hard, hard_geo, hard_cap, d, eps, dt, ct, ct_s, ct_vol, ct_grad, ct_cap,
                                           pair_cnt, nullptr, 0.0f, cnt);
  }
}

}  // namespace stiv
