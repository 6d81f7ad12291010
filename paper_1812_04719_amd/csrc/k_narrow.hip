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
// edge, at both ends of the step, over the mean edge length at t_n).  The
// search then certifies [0, lo) root-free with one Bernstein test and looks
// in [lo, hi] first (earliest_bracket in narrow_math.h); the contacts found
// are the same as without the prediction.
#include "mlp_tile.h"
#include "narrow_math.h"

namespace stiv {

namespace {

using namespace nm;

__device__ inline unsigned long long lanemask_lt() {
  const int lane = threadIdx.x & 63;
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ inline d3 load_pos(const double *x, int64_t nv, int64_t gid) {
  return mk(x[gid], x[nv + gid], x[2 * nv + gid]);
}

// Global vertex ids and per-vertex image shifts of a candidate; order
// (p, a, b, c) for vertex-triangle, (a, b, c, e) for edge-edge.  side[k] is 1
// for vertices of the pair's second vesicle (shifted by sigma L).
__device__ inline void cand_vertices(const DevScene &S, const DevTopo &T, const PairRec &pr, const Cand &c,
                                     int64_t gid[4], int side[4]) {
  if (c.kind == 2) {
    const int ta = S.topo_id[pr.a], tb = S.topo_id[pr.b];
    const int *ea = T.edge + 2 * ((int64_t)T.edge_off[ta] + c.i);
    const int *eb = T.edge + 2 * ((int64_t)T.edge_off[tb] + c.j);
    gid[0] = S.vtx_off[pr.a] + ea[0]; gid[1] = S.vtx_off[pr.a] + ea[1];
    gid[2] = S.vtx_off[pr.b] + eb[0]; gid[3] = S.vtx_off[pr.b] + eb[1];
    side[0] = side[1] = 0; side[2] = side[3] = 1;
  } else {
    const int vv = c.kind ? pr.b : pr.a, vt = c.kind ? pr.a : pr.b;
    const int *tri = T.tri + 3 * ((int64_t)T.tri_off[S.topo_id[vt]] + c.j);
    gid[0] = S.vtx_off[vv] + c.i;
    for (int q = 0; q < 3; ++q) gid[1 + q] = S.vtx_off[vt] + tri[q];
    side[0] = c.kind ? 1 : 0;
    side[1] = side[2] = side[3] = c.kind ? 0 : 1;
  }
}

// Load the candidate's vertices; Q gets X0 + shift and D = X1 - X0.  Returns
// whether the FP64 primitive boxes overlap, box = ((min over the primitive's
// vertices of min(X0, X1)) - h) + shift, likewise for the max.  The first
// primitive is vertex 0 (vertex-triangle) or vertices 0-1 (edge-edge); the
// second is vertices 1-3 or 2-3.
__device__ inline bool load_quad(const DevScene &S, const PairRec &pr, const int64_t gid[4], const int side[4],
                                 bool ee, double h, Quad &Q) {
  const int64_t NV = S.n_vtx;
  d3 a[4], b[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    a[k] = load_pos(S.x0, NV, gid[k]);
    b[k] = load_pos(S.x1, NV, gid[k]);
    const double sx = side[k] ? pr.sh[0] : 0.0, sy = side[k] ? pr.sh[1] : 0.0, sz = side[k] ? pr.sh[2] : 0.0;
    Q.X0[k] = mk(a[k].x + sx, a[k].y + sy, a[k].z + sz);
    Q.D[k] = b[k] - a[k];
  }
  Q.ee = ee;
  const d3 lo0 = vmin(a[0], b[0]), hi0 = vmax(a[0], b[0]);
  const d3 lo1 = vmin(a[1], b[1]), hi1 = vmax(a[1], b[1]);
  const d3 lo2 = vmin(vmin(a[2], b[2]), vmin(a[3], b[3])), hi2 = vmax(vmax(a[2], b[2]), vmax(a[3], b[3]));
  // vertex 1 belongs to the first primitive for edge-edge, to the triangle otherwise
  const d3 lA = ee ? vmin(lo0, lo1) : lo0, hA = ee ? vmax(hi0, hi1) : hi0;
  const d3 lB = ee ? lo2 : vmin(lo1, lo2), hB = ee ? hi2 : vmax(hi1, hi2);
  const d3 sA = side[0] ? mk(pr.sh[0], pr.sh[1], pr.sh[2]) : mk(0.0, 0.0, 0.0);
  const d3 sB = side[3] ? mk(pr.sh[0], pr.sh[1], pr.sh[2]) : mk(0.0, 0.0, 0.0);
  const d3 l0 = (lA - mk(h, h, h)) + sA, u0 = (hA + mk(h, h, h)) + sA;
  const d3 l1 = (lB - mk(h, h, h)) + sB, u1 = (hB + mk(h, h, h)) + sB;
  return l0.x <= u1.x && l1.x <= u0.x && l0.y <= u1.y && l1.y <= u0.y && l0.z <= u1.z && l1.z <= u0.z;
}

__device__ inline double len3(const d3 &v) { return sqrt(dotp(v, v)); }

// Features of the learned bracket from the candidate's positions (selects,
// not indices, pick the vertices so that Q stays in registers).
__device__ inline void bracket_features(const Quad &Q, float out[mlp::kIn]) {
  const bool ee = Q.ee;
  double ell;
  if (ee) {
    ell = 0.5 * (len3(Q.X0[1] - Q.X0[0]) + len3(Q.X0[3] - Q.X0[2]));
  } else {
    ell = (len3(Q.X0[2] - Q.X0[1]) + len3(Q.X0[3] - Q.X0[1]) + len3(Q.X0[3] - Q.X0[2])) / 3.0;
  }
  const double inv = ell > 0.0 ? 1.0 / ell : 1.0;
  const d3 A0 = ee ? Q.X0[0] : Q.X0[1], AD = ee ? Q.D[0] : Q.D[1];
  const d3 P0[3] = {ee ? Q.X0[1] : Q.X0[2], ee ? Q.X0[2] : Q.X0[3], ee ? Q.X0[3] : Q.X0[0]};
  const d3 PD[3] = {ee ? Q.D[1] : Q.D[2], ee ? Q.D[2] : Q.D[3], ee ? Q.D[3] : Q.D[0]};
  const d3 A1 = A0 + AD;
#pragma unroll
  for (int r = 0; r < 3; ++r) {
    const d3 a = P0[r] - A0;
    const d3 b = (P0[r] + PD[r]) - A1;
    out[3 * r + 0] = (float)(a.x * inv);
    out[3 * r + 1] = (float)(a.y * inv);
    out[3 * r + 2] = (float)(a.z * inv);
    out[9 + 3 * r + 0] = (float)(b.x * inv);
    out[9 + 3 * r + 1] = (float)(b.y * inv);
    out[9 + 3 * r + 2] = (float)(b.z * inv);
  }
}

struct BracketLds {
  mlp::Weights W;
  unsigned short x[256][mlp::kInP];
  mlp::Act act[4];
  float br[256][2];
};

// Root search on the queued candidates, then volume and gradient on contact.
// LEARNED: the bracket of every candidate is predicted first (all 256
// candidates of the workgroup through the perceptron on the matrix cores).
template <int N, bool LEARNED>
__global__ __launch_bounds__(256) void k_narrow(DevScene S, DevTopo T, const PairRec *pairs, const Cand *hard,
                                                int64_t hard_cap, double d, double eps,
                                                double dt, Cand *ct, double *ct_s, double *ct_vol, double *ct_grad,
                                                int64_t ct_cap, const float *mlp_params, float kwidth,
                                                Counters *cnt) {
  int64_t nc = (int64_t)cnt->n_hard;
  nc = nc < hard_cap ? nc : hard_cap;
  int within = 0, deg = 0, cert = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  extern __shared__ char dyn_lds[];
  BracketLds &L = *reinterpret_cast<BracketLds *>(dyn_lds);
  if (LEARNED) {
    if ((int64_t)blockIdx.x * blockDim.x >= nc) return;  // whole workgroup idle: uniform exit
    mlp::stage_weights(L.W, mlp_params);
  }
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nc; base += stride) {
    const int64_t i = base + threadIdx.x;
    int hit = 0;
    double s = 0.0, V = 0.0, g[12];
    Cand c;
    c.pair = c.kind = c.i = c.j = 0;
    for (int k = 0; k < 12; ++k) g[k] = 0.0;
    Quad Q;
    PairRec pr;
    int64_t gid[4];
    int side[4];
    if (i < nc) {
      c = hard[i];
      pr = pairs[c.pair];
      cand_vertices(S, T, pr, c, gid, side);
    }
    if (LEARNED) {
      // features first; the positions are loaded again for the search so that
      // they are not live (spilled) across the perceptron
      {
        float ft[mlp::kIn];
        if (i < nc) {
          Quad Qf;
          load_quad(S, pr, gid, side, c.kind == 2, 0.5 * d, Qf);
          bracket_features(Qf, ft);
        } else {
#pragma unroll
          for (int k = 0; k < mlp::kIn; ++k) ft[k] = 0.0f;
        }
#pragma unroll
        for (int k = 0; k < mlp::kInP; ++k) L.x[threadIdx.x][k] = k < mlp::kIn ? mlp::f2bf(ft[k]) : 0;
      }
      __syncthreads();
      const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
      for (int q = 0; q < 4; ++q) {
        const int row0 = 64 * wave + 16 * q;
        const mlp::f32x4 o = mlp::forward16(L.W, &L.x[row0][0], L.act[wave]);
        const int col = lane & 15, gq = lane >> 4;
        if (col < 2)
          for (int j = 0; j < 4; ++j) L.br[row0 + 4 * gq + j][col] = o[j];
        __syncthreads();
      }
      if (i < nc) {
        load_quad(S, pr, gid, side, c.kind == 2, 0.5 * d, Q);
        const float mu = mlp::head_mu(L.br[threadIdx.x][0]), sd = mlp::head_sd(L.br[threadIdx.x][1]);
        double lo = (double)mu - (double)kwidth * (double)sd, hi = (double)mu + (double)kwidth * (double)sd;
        lo = lo < 0.0 ? 0.0 : lo;
        hi = hi > 1.0 ? 1.0 : hi;
        int certified = 0;
        hit = earliest_bracket<N>(Q, d, lo, hi, &s, &within, &deg, &certified);
        cert += certified;
      }
      __syncthreads();
    } else if (i < nc) {
      load_quad(S, pr, gid, side, c.kind == 2, 0.5 * d, Q);
      hit = earliest<N>(Q, d, &s, &within, &deg);
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
    if (hit) {
      const unsigned long long slot = slot0 + __popcll(m & lanemask_lt());
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
  if (LEARNED && cert) atomicAdd(&cnt->n_bracket_ok, (unsigned long long)cert);
}

}  // namespace

static int grid_for(int64_t n, int max_blocks) {
  int64_t g = (n + 255) / 256;
  if (g > max_blocks) g = max_blocks;
  if (g < 1) g = 1;
  return (int)g;
}

void launch_narrow(int blocks, const DevScene &S, const DevTopo &T, const PairRec *pairs, const Cand *hard, int64_t hard_cap,
                   double d, double eps, double dt, Cand *ct, double *ct_s, double *ct_vol, double *ct_grad,
                   int64_t ct_cap, const float *mlp_params, float kwidth, Counters *cnt, hipStream_t st) {
  const int g = grid_for(hard_cap, blocks);
  const size_t lds = sizeof(BracketLds);
  if (mlp_params) {
    if (d == 0.0)
      k_narrow<3, true><<<g, 256, lds, st>>>(S, T, pairs, hard, hard_cap, d, eps, dt, ct, ct_s, ct_vol, ct_grad, ct_cap,
                                            mlp_params, kwidth, cnt);
    else
      k_narrow<6, true><<<g, 256, lds, st>>>(S, T, pairs, hard, hard_cap, d, eps, dt, ct, ct_s, ct_vol, ct_grad, ct_cap,
                                            mlp_params, kwidth, cnt);
  } else {
    if (d == 0.0)
      k_narrow<3, false><<<g, 256, 0, st>>>(S, T, pairs, hard, hard_cap, d, eps, dt, ct, ct_s, ct_vol, ct_grad, ct_cap,
                                           nullptr, 0.0f, cnt);
    else
      k_narrow<6, false><<<g, 256, 0, st>>>(S, T, pairs, hard, hard_cap, d, eps, dt, ct, ct_s, ct_vol, ct_grad, ct_cap,
                                           nullptr, 0.0f, cnt);
  }
}

}  // namespace stiv
