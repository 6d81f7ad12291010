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

// Bisection on [lo, hi] with f(lo) = flo != 0 and a sign change; width 2^-50.
__host__ __device__ double refine(const double f[7], int n, double lo, double hi, double flo) {
  const double tol = 8.881784197001252e-16;
  for (int it = 0; it < 120 && hi - lo > tol; ++it) {
    const double mid = 0.5 * (lo + hi);
    const double fm = horner(f, n, mid);
    if (fm == 0.0) return mid;
    if ((fm < 0.0) == (flo < 0.0)) { lo = mid; flo = fm; } else hi = mid;
  }
  return 0.5 * (lo + hi);
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

__global__ __launch_bounds__(256) void k_narrow(DevScene S, DevTopo T, const PairRec *pairs, const Cand *cand,
                                                int64_t cand_cap, double d, double eps, double dt, Cand *ct,
                                                double *ct_s, double *ct_vol, double *ct_grad, int64_t ct_cap,
                                                Counters *cnt) {
  int64_t nc = (int64_t)cnt->n_cand;
  nc = nc < cand_cap ? nc : cand_cap;
  const int64_t NV = S.n_vtx;
  int within = 0, deg = 0;
  // uniform trip count per wavefront so the ballot below sees every lane
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < nc; base += stride) {
    const int64_t i = base + threadIdx.x;
    int hit = 0;
    double s = 0.0, V = 0.0, g[12];
    Cand c;
    c.pair = c.kind = c.i = c.j = 0;
    for (int k = 0; k < 12; ++k) g[k] = 0.0;
    if (i < nc) {
      c = cand[i];
      const PairRec pr = pairs[c.pair];
      int64_t gid[4];
      double shk[4][3];
      Quad Q;
      Q.ee = (c.kind == 2);
      if (c.kind == 2) {
        const int ta = S.topo_id[pr.a], tb = S.topo_id[pr.b];
        const int *ea = T.edge + 2 * ((int64_t)T.edge_off[ta] + c.i);
        const int *eb = T.edge + 2 * ((int64_t)T.edge_off[tb] + c.j);
        gid[0] = S.vtx_off[pr.a] + ea[0]; gid[1] = S.vtx_off[pr.a] + ea[1];
        gid[2] = S.vtx_off[pr.b] + eb[0]; gid[3] = S.vtx_off[pr.b] + eb[1];
        for (int q = 0; q < 3; ++q) {
          shk[0][q] = shk[1][q] = 0.0;
          shk[2][q] = shk[3][q] = pr.sh[q];
        }
      } else {
        const int vv = c.kind ? pr.b : pr.a, vt = c.kind ? pr.a : pr.b;
        const int tt = S.topo_id[vt];
        const int *tri = T.tri + 3 * ((int64_t)T.tri_off[tt] + c.j);
        gid[0] = S.vtx_off[vv] + c.i;
        for (int q = 0; q < 3; ++q) gid[1 + q] = S.vtx_off[vt] + tri[q];
        for (int q = 0; q < 3; ++q) {
          const double sv = c.kind ? pr.sh[q] : 0.0, st = c.kind ? 0.0 : pr.sh[q];
          shk[0][q] = sv;
          shk[1][q] = shk[2][q] = shk[3][q] = st;
        }
      }
      for (int k = 0; k < 4; ++k) {
        const d3 a = load_pos(S.x0, NV, gid[k]), b = load_pos(S.x1, NV, gid[k]);
        Q.X0[k] = mk(a.x + shk[k][0], a.y + shk[k][1], a.z + shk[k][2]);
        Q.D[k] = b - a;
      }
      hit = earliest(Q, d, &s, &within, &deg);
      if (hit && !Q.ee) volume_grad(Q, s, d, eps, dt, s == 0.0, &V, g);
    }
    const unsigned long long m = __ballot(hit != 0);
    const int nh = __popcll(m);
    unsigned long long slot0 = 0;
    const int leader = m ? __ffsll((long long)m) - 1 : 0;
    const int nee_w = __popcll(__ballot(hit != 0 && c.kind == 2));
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

void launch_narrow(const DevScene &S, const DevTopo &T, const PairRec *pairs, const Cand *cand, int64_t cand_cap,
                   double d, double eps, double dt, Cand *ct, double *ct_s, double *ct_vol, double *ct_grad,
                   int64_t ct_cap, Counters *cnt, hipStream_t st) {
  int64_t g = (cand_cap + 255) / 256;
  if (g > 4096) g = 4096;
  if (g < 1) g = 1;
  k_narrow<<<(int)g, 256, 0, st>>>(S, T, pairs, cand, cand_cap, d, eps, dt, ct, ct_s, ct_vol, ct_grad, ct_cap, cnt);
}

}  // namespace stiv
