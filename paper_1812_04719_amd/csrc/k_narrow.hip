// K3 + K4: narrow phase (Eq. 3.1) and contact volume with its gradient
// (Eq. 3.2, App. A), FP64, one thread per primitive candidate.
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
#include "stiv_common.h"

namespace stiv {

namespace {

struct d3 {
  double x, y, z;
};
__host__ __device__ inline d3 mk(double x, double y, double z) { return d3{x, y, z}; }
__host__ __device__ inline d3 operator+(d3 a, d3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
__host__ __device__ inline d3 operator-(d3 a, d3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
__host__ __device__ inline d3 operator*(double s, d3 a) { return mk(s * a.x, s * a.y, s * a.z); }
__host__ __device__ inline double dotp(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__host__ __device__ inline d3 crossp(d3 a, d3 b) {
  return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

struct Quad {
  d3 X0[4], D[4];  // vertex-triangle: p, a, b, c; edge-edge: a, b, c, e
  bool ee;
};

__host__ __device__ inline d3 at(const Quad &Q, int k, double s) { return Q.X0[k] + s * Q.D[k]; }

// F coefficients, lowest degree first; returns the degree (6, or 3 if d == 0).
__host__ __device__ int poly_coeffs(const Quad &Q, double d, double f[7]) {
  d3 u0, u1, v0, v1, w0, w1;
  if (!Q.ee) {
    u0 = Q.X0[2] - Q.X0[1]; u1 = Q.D[2] - Q.D[1];
    v0 = Q.X0[3] - Q.X0[1]; v1 = Q.D[3] - Q.D[1];
    w0 = Q.X0[0] - Q.X0[1]; w1 = Q.D[0] - Q.D[1];
  } else {
    u0 = Q.X0[1] - Q.X0[0]; u1 = Q.D[1] - Q.D[0];
    v0 = Q.X0[3] - Q.X0[2]; v1 = Q.D[3] - Q.D[2];
    w0 = Q.X0[2] - Q.X0[0]; w1 = Q.D[2] - Q.D[0];
  }
  const d3 n0 = crossp(u0, v0);
  const d3 n1 = crossp(u0, v1) + crossp(u1, v0);
  const d3 n2 = crossp(u1, v1);
  const double g0 = dotp(w0, n0), g1 = dotp(w1, n0) + dotp(w0, n1), g2 = dotp(w1, n1) + dotp(w0, n2),
               g3 = dotp(w1, n2);
  if (d == 0.0) {
    f[0] = g0; f[1] = g1; f[2] = g2; f[3] = g3;
    f[4] = f[5] = f[6] = 0.0;
    return 3;
  }
  const double q0 = dotp(n0, n0), q1 = 2.0 * dotp(n0, n1), q2 = dotp(n1, n1) + 2.0 * dotp(n0, n2),
               q3 = 2.0 * dotp(n1, n2), q4 = dotp(n2, n2);
  const double dd = d * d;
  f[0] = g0 * g0 - dd * q0;
  f[1] = 2.0 * (g0 * g1) - dd * q1;
  f[2] = (g1 * g1 + 2.0 * (g0 * g2)) - dd * q2;
  f[3] = 2.0 * (g0 * g3 + g1 * g2) - dd * q3;
  f[4] = (g2 * g2 + 2.0 * (g1 * g3)) - dd * q4;
  f[5] = 2.0 * (g2 * g3);
  f[6] = g3 * g3;
  return 6;
}

__host__ __device__ inline double horner(const double f[7], int n, double s) {
  double r = f[n];
  for (int k = n - 1; k >= 0; --k) r = r * s + f[k];
  return r;
}

// 1 inside, 0 outside, -1 degenerate (normal vanishes).
__host__ __device__ int inside_at(const Quad &Q, double s) {
  const d3 A = at(Q, 0, s), B = at(Q, 1, s), C = at(Q, 2, s), E = at(Q, 3, s);
  if (!Q.ee) {
    const d3 e1 = C - B, e2 = E - B, w = A - B;
    const d3 n = crossp(e1, e2);
    const double q = dotp(n, n);
    if (q == 0.0) return -1;
    const double bb = dotp(crossp(w, e2), n), cc = dotp(crossp(e1, w), n);
    return (bb >= 0.0 && cc >= 0.0 && bb + cc <= q) ? 1 : 0;
  }
  const d3 ea = B - A, eb = E - C, w = C - A;
  const d3 m = crossp(ea, eb);
  const double q = dotp(m, m);
  if (q == 0.0) return -1;
  const double uu = dotp(crossp(w, eb), m), vv = dotp(crossp(w, ea), m);
  return (uu >= 0.0 && uu <= q && vv >= 0.0 && vv <= q) ? 1 : 0;
}

// Bernstein coefficients of f restricted to [u, u + wd], written in place of b.
__host__ __device__ void bernstein_on(const double f[7], int n, double u, double wd, double b[7]) {
  double c[7];
  for (int k = 0; k <= n; ++k) c[k] = f[k];
  // Taylor shift to u: c(x) = f(u + x)
  for (int i = 0; i < n; ++i)
    for (int k = n - 1; k >= i; --k) c[k] += u * c[k + 1];
  // scale x = wd t
  double p = wd;
  for (int k = 1; k <= n; ++k) { c[k] *= p; p *= wd; }
  // power -> Bernstein: b_j = sum_{k<=j} C(j,k)/C(n,k) c_k
  // Pascal-like recurrence: repeatedly b_j += b_{j-1} with weights, done via
  // the standard triangular scheme on c_k / C(n,k).
  double binom_n[7] = {1, 0, 0, 0, 0, 0, 0};
  for (int k = 1; k <= n; ++k) binom_n[k] = binom_n[k - 1] * (double)(n - k + 1) / (double)k;
  for (int k = 0; k <= n; ++k) c[k] /= binom_n[k];
  // b_j = sum_k C(j,k) c'_k : apply j-fold prefix summation
  for (int j = 0; j <= n; ++j) b[j] = c[j];
  for (int r = 1; r <= n; ++r)
    for (int j = n; j >= r; --j) b[j] += b[j - 1];
}

// Root of f in [lo, hi] where f(lo) = flo != 0 and f changes sign: Newton
// steps kept inside the shrinking bracket, bisection when a step would leave
// it or converge too slowly; stops at a step below 2^-52 or a bracket of
// width 2^-50.
__host__ __device__ double refine(const double f[7], int n, double lo, double hi, double flo) {
  const double tol = 8.881784197001252e-16;
  double x = 0.5 * (lo + hi), dx = hi - lo, dxold = dx;
  for (int it = 0; it < 100; ++it) {
    double fx = f[n], dfx = 0.0;
    for (int k = n - 1; k >= 0; --k) {
      dfx = dfx * x + fx;
      fx = fx * x + f[k];
    }
    if (fx == 0.0) return x;
    if ((fx < 0.0) == (flo < 0.0)) { lo = x; flo = fx; } else { hi = x; }
    if (hi - lo <= tol) break;
    const double xn = (dfx != 0.0) ? x - fx / dfx : x;
    if (!(xn > lo && xn < hi) || fabs(2.0 * fx) > fabs(dxold * dfx)) {
      dxold = dx;
      dx = 0.5 * (hi - lo);
      x = lo + dx;
    } else {
      dxold = dx;
      dx = xn - x;
      x = xn;
      if (fabs(dx) <= 2.220446049250313e-16 * fmax(fabs(x), 1e-300)) break;
    }
  }
  return x;
}

// Earliest valid root.  Returns 1 with *s on contact, 0 otherwise.
// *deg counts degenerate skips (vanishing normal at a root, or F == 0).
__host__ __device__ int earliest(const Quad &Q, double d, double *s_out, int *within, int *deg) {
  double f[7];
  const int n = poly_coeffs(Q, d, f);
  bool allzero = true;
  for (int k = 0; k <= n; ++k) allzero &= (f[k] == 0.0);
  if (allzero) { (*deg)++; return 0; }
  if (d > 0.0 && f[0] < 0.0 && inside_at(Q, 0.0) == 1) {
    (*within)++;
    *s_out = 0.0;
    return 1;
  }
  const int kMaxLevel = 44;
  // Bound on visited intervals: a well-posed sextic needs a few dozen; a
  // polynomial that is zero up to rounding over a whole interval would
  // otherwise make the traversal exponential.  Such inputs are reported as
  // degenerate.
  const int kMaxVisits = 4096;
  int level = 0, visits = 0;
  long long idx = 0;
  while (true) {
    if (++visits > kMaxVisits) {
      (*deg)++;
      return 0;
    }
    const double wd = ldexp(1.0, -level);
    const double u = (double)idx * wd;
    double b[7];
    bernstein_on(f, n, u, wd, b);
    bool pos = true, neg = true;
    int changes = 0, last = 0;
    for (int k = 0; k <= n; ++k) {
      pos &= b[k] > 0.0;
      neg &= b[k] < 0.0;
      const int sg = (b[k] > 0.0) - (b[k] < 0.0);
      if (sg != 0) {
        if (last != 0 && sg != last) ++changes;
        last = sg;
      }
    }
    bool descend = false;
    if (!(pos || neg)) {
      const double v = u + wd;
      const double fu = horner(f, n, u), fv = horner(f, n, v);
      double root = -1.0;
      if (changes == 1 && b[0] != 0.0 && b[n] != 0.0 && fu != 0.0 && fv != 0.0 && ((fu < 0.0) != (fv < 0.0))) {
        root = refine(f, n, u, v, fu);
      } else if (level < kMaxLevel) {
        descend = true;
      } else if (fu == 0.0) {
        root = u;
      } else if (fv != 0.0 && ((fu < 0.0) != (fv < 0.0))) {
        root = refine(f, n, u, v, fu);
      }
      if (root >= 0.0) {
        const int in = inside_at(Q, root);
        if (in < 0) (*deg)++;
        if (in == 1) {
          *s_out = root;
          return 1;
        }
      }
    }
    if (descend) {
      ++level;
      idx <<= 1;
      continue;
    }
    // next interval in left-to-right order
    while (level > 0 && (idx & 1)) { idx >>= 1; --level; }
    if (level == 0) break;
    ++idx;
  }
  return 0;
}

// V and dV/dX1 (order p, a, b, c) of a vertex-triangle contact at s.
__host__ __device__ void volume_grad(const Quad &Q, double s, double d, double eps, double dt, bool clamped, double *V,
                            double g[12]) {
  const d3 Pp = at(Q, 0, s), Pa = at(Q, 1, s), Pb = at(Q, 2, s), Pc = at(Q, 3, s);
  const d3 e1 = Pb - Pa, e2 = Pc - Pa, w = Pp - Pa;
  const d3 e1s = Q.D[2] - Q.D[1], e2s = Q.D[3] - Q.D[1], ws = Q.D[0] - Q.D[1];
  const d3 n = crossp(e1, e2);
  const double q = dotp(n, n);
  const d3 U = (1.0 / dt) * Q.D[0];
  const double un = dotp(U, n);
  const double R = sqrt(eps * eps * q + un * un);
  *V = 0.5 * dt * (1.0 - s) * R;
  const d3 m = (1.0 / R) * ((eps * eps) * n + un * U);
  const double k = 0.5 * dt * (1.0 - s);
  d3 gp = (0.5 * (1.0 - s) * un / R) * n;
  d3 ga = (k * s) * crossp(e1 - e2, m);
  d3 gb = (k * s) * crossp(e2, m);
  d3 gc = (k * s) * crossp(m, e1);
  if (!clamped) {
    const d3 ns = crossp(e1s, e2) + crossp(e1, e2s);
    const double gv = dotp(w, n);
    const double gs = dotp(ws, n) + dotp(w, ns);
    const d3 dgp = n, dga = crossp(e1 - e2, w) - n, dgb = crossp(e2, w), dgc = crossp(w, e1);
    double Fs;
    d3 Fp, Fa, Fb, Fc;
    if (d == 0.0) {
      Fs = gs; Fp = dgp; Fa = dga; Fb = dgb; Fc = dgc;
    } else {
      const double dd = d * d;
      Fs = 2.0 * gv * gs - 2.0 * dd * dotp(n, ns);
      Fp = (2.0 * gv) * dgp;
      Fa = (2.0 * gv) * dga - dd * (2.0 * crossp(e1 - e2, n));
      Fb = (2.0 * gv) * dgb - dd * (2.0 * crossp(e2, n));
      Fc = (2.0 * gv) * dgc - dd * (2.0 * crossp(n, e1));
    }
    if (Fs != 0.0) {
      const double dVds = 0.5 * dt * (-R + (1.0 - s) * dotp(m, ns));
      const double cf = -dVds * s / Fs;
      gp = gp + cf * Fp;
      ga = ga + cf * Fa;
      gb = gb + cf * Fb;
      gc = gc + cf * Fc;
    }
  }
  g[0] = gp.x; g[1] = gp.y; g[2] = gp.z;
  g[3] = ga.x; g[4] = ga.y; g[5] = ga.z;
  g[6] = gb.x; g[7] = gb.y; g[8] = gb.z;
  g[9] = gc.x; g[10] = gc.y; g[11] = gc.z;
}

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

// Load the candidate's vertices; Q gets X0 + shift and D = X1 - X0, raw the
// unshifted positions.  Returns whether the FP64 primitive boxes overlap:
// box = ((min over vertices of min(X0, X1)) - h) + shift, likewise for max.
__device__ inline bool load_quad(const DevScene &S, const PairRec &pr, const int64_t gid[4], const int side[4],
                                 bool ee, double h, Quad &Q) {
  const int64_t NV = S.n_vtx;
  double lo[2][3], hi[2][3];
  for (int g = 0; g < 2; ++g)
    for (int c = 0; c < 3; ++c) { lo[g][c] = INFINITY; hi[g][c] = -INFINITY; }
  Q.ee = ee;
  for (int k = 0; k < 4; ++k) {
    const d3 a = load_pos(S.x0, NV, gid[k]), b = load_pos(S.x1, NV, gid[k]);
    const double sx = side[k] ? pr.sh[0] : 0.0, sy = side[k] ? pr.sh[1] : 0.0, sz = side[k] ? pr.sh[2] : 0.0;
    Q.X0[k] = mk(a.x + sx, a.y + sy, a.z + sz);
    Q.D[k] = b - a;
    // group 0: first primitive (vertex, or edge a-b); group 1: triangle or edge c-e
    const int grp = ee ? (k >= 2) : (k >= 1);
    lo[grp][0] = fmin(lo[grp][0], fmin(a.x, b.x)); hi[grp][0] = fmax(hi[grp][0], fmax(a.x, b.x));
    lo[grp][1] = fmin(lo[grp][1], fmin(a.y, b.y)); hi[grp][1] = fmax(hi[grp][1], fmax(a.y, b.y));
    lo[grp][2] = fmin(lo[grp][2], fmin(a.z, b.z)); hi[grp][2] = fmax(hi[grp][2], fmax(a.z, b.z));
  }
  // shift of each group (all vertices of a group are on the same side)
  const int sg0 = side[0], sg1 = side[3];
  bool ov = true;
  for (int c = 0; c < 3; ++c) {
    const double s0 = sg0 ? pr.sh[c] : 0.0, s1 = sg1 ? pr.sh[c] : 0.0;
    const double l0 = (lo[0][c] - h) + s0, u0 = (hi[0][c] + h) + s0;
    const double l1 = (lo[1][c] - h) + s1, u1 = (hi[1][c] + h) + s1;
    ov = ov && (l0 <= u1) && (l1 <= u0);
  }
  return ov;
}

// Screen: exact box test (counts the candidate), polynomial coefficients and
// one Bernstein test on [0,1].  A polynomial with all Bernstein coefficients
// positive (d > 0), or of one strict sign (d = 0), has no root and no
// within-d start; everything else goes to the root search queue.
__global__ __launch_bounds__(256) void k_narrow_screen(DevScene S, DevTopo T, const PairRec *pairs,
                                                       const Cand *pre, int64_t pre_cap, double d, int32_t *hard,
                                                       int64_t hard_cap, Cand *list, int64_t list_cap,
                                                       Counters *cnt) {
  int64_t n = (int64_t)cnt->n_pre;
  n = n < pre_cap ? n : pre_cap;
  const double h = 0.5 * d;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  unsigned long long nvt = 0, nee = 0;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < n; base += stride) {
    const int64_t i = base + threadIdx.x;
    bool is_cand = false, need = false;
    Cand c;
    c.pair = c.kind = c.i = c.j = 0;
    if (i < n) {
      c = pre[i];
      const PairRec pr = pairs[c.pair];
      int64_t gid[4];
      int side[4];
      cand_vertices(S, T, pr, c, gid, side);
      Quad Q;
      is_cand = load_quad(S, pr, gid, side, c.kind == 2, h, Q);
      if (is_cand) {
        if (c.kind == 2) ++nee; else ++nvt;
        double f[7], b[7];
        const int deg = poly_coeffs(Q, d, f);
        bernstein_on(f, deg, 0.0, 1.0, b);
        bool pos = true, neg = true;
        for (int k = 0; k <= deg; ++k) { pos &= b[k] > 0.0; neg &= b[k] < 0.0; }
        need = !(pos || (d == 0.0 && neg));
      }
    }
    const unsigned long long mh = __ballot(need);
    const int leader_h = mh ? __ffsll((long long)mh) - 1 : 0;
    unsigned long long bh = 0;
    if ((int)(threadIdx.x & 63) == leader_h && mh) bh = atomicAdd(&cnt->n_hard, (unsigned long long)__popcll(mh));
    bh = __shfl(bh, leader_h, 64);
    if (need) {
      const unsigned long long slot = bh + __popcll(mh & lanemask_lt());
      if ((int64_t)slot < hard_cap) hard[slot] = (int32_t)i;
    }
    if (list) {
      const unsigned long long mc = __ballot(is_cand);
      const int leader_c = mc ? __ffsll((long long)mc) - 1 : 0;
      unsigned long long bc = 0;
      if ((int)(threadIdx.x & 63) == leader_c && mc)
        bc = atomicAdd(&cnt->n_cand_list, (unsigned long long)__popcll(mc));
      bc = __shfl(bc, leader_c, 64);
      if (is_cand) {
        const unsigned long long slot = bc + __popcll(mc & lanemask_lt());
        if ((int64_t)slot < list_cap) list[slot] = c;
      }
    }
  }
  // one atomic per wavefront for the candidate counts
  for (int off = 32; off > 0; off >>= 1) {
    nvt += __shfl_xor(nvt, off, 64);
    nee += __shfl_xor(nee, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    if (nvt) atomicAdd(&cnt->n_cand_vt, nvt);
    if (nee) atomicAdd(&cnt->n_cand_ee, nee);
  }
}

// Root search on the queued candidates, then volume and gradient on contact.
__global__ __launch_bounds__(256) void k_narrow(DevScene S, DevTopo T, const PairRec *pairs, const Cand *pre,
                                                const int32_t *hard, int64_t hard_cap, double d, double eps,
                                                double dt, Cand *ct, double *ct_s, double *ct_vol, double *ct_grad,
                                                int64_t ct_cap, Counters *cnt) {
  int64_t nc = (int64_t)cnt->n_hard;
  nc = nc < hard_cap ? nc : hard_cap;
  int within = 0, deg = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nc; base += stride) {
    const int64_t i = base + threadIdx.x;
    int hit = 0;
    double s = 0.0, V = 0.0, g[12];
    Cand c;
    c.pair = c.kind = c.i = c.j = 0;
    for (int k = 0; k < 12; ++k) g[k] = 0.0;
    if (i < nc) {
      c = pre[hard[i]];
      const PairRec pr = pairs[c.pair];
      int64_t gid[4];
      int side[4];
      cand_vertices(S, T, pr, c, gid, side);
      Quad Q;
      load_quad(S, pr, gid, side, c.kind == 2, 0.5 * d, Q);
      hit = earliest(Q, d, &s, &within, &deg);
      if (hit && !Q.ee) volume_grad(Q, s, d, eps, dt, s == 0.0, &V, g);
    }
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
}

}  // namespace

static int grid_for(int64_t n) {
  int64_t g = (n + 255) / 256;
  if (g > 8192) g = 8192;
  if (g < 1) g = 1;
  return (int)g;
}

void launch_narrow_screen(const DevScene &S, const DevTopo &T, const PairRec *pairs, const Cand *pre,
                          int64_t pre_cap, double d, int32_t *hard, int64_t hard_cap, Cand *list, int64_t list_cap,
                          Counters *cnt, hipStream_t st) {
  k_narrow_screen<<<grid_for(pre_cap), 256, 0, st>>>(S, T, pairs, pre, pre_cap, d, hard, hard_cap, list, list_cap,
                                                     cnt);
}

void launch_narrow(const DevScene &S, const DevTopo &T, const PairRec *pairs, const Cand *pre, const int32_t *hard,
                   int64_t hard_cap, double d, double eps, double dt, Cand *ct, double *ct_s, double *ct_vol,
                   double *ct_grad, int64_t ct_cap, Counters *cnt, hipStream_t st) {
  k_narrow<<<grid_for(hard_cap), 256, 0, st>>>(S, T, pairs, pre, hard, hard_cap, d, eps, dt, ct, ct_s, ct_vol,
                                               ct_grad, ct_cap, cnt);
}

}  // namespace stiv
