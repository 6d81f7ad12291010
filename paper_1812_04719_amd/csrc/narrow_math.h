// FP64 narrow-phase mathematics shared by the primitive-candidate kernel
// (screen) and the root-search kernel.  See k_narrow.hip for the method.
#pragma once
#include "stiv_common.h"

namespace stiv {
namespace nm {

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
__host__ __device__ inline d3 vmin(d3 a, d3 b) { return mk(fmin(a.x, b.x), fmin(a.y, b.y), fmin(a.z, b.z)); }
__host__ __device__ inline d3 vmax(d3 a, d3 b) { return mk(fmax(a.x, b.x), fmax(a.y, b.y), fmax(a.z, b.z)); }

// F coefficients, lowest degree first.  N = 6: F = g^2 - d^2 q; N = 3: F = g
// (used when d == 0).  All loops have compile-time bounds so the coefficient
// arrays stay in registers.
template <int N>
__host__ __device__ void poly_coeffs(const Quad &Q, double d, double f[N + 1]) {
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
  if constexpr (N == 3) {
    (void)d;
    f[0] = g0; f[1] = g1; f[2] = g2; f[3] = g3;
  } else {
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
  }
}

template <int N>
__host__ __device__ inline double horner(const double f[N + 1], double s) {
  double r = f[N];
#pragma unroll
  for (int k = N - 1; k >= 0; --k) r = r * s + f[k];
  return r;
}

// 1 inside, 0 outside, -1 degenerate (normal vanishes).
__host__ __device__ inline int inside_at(const Quad &Q, double s) {
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

// Positive multiples of Bernstein coefficients.  The coefficients in the
// Bernstein basis are b_j = sum_{k<=j} C(j,k)/C(N,k) c_k (j-fold prefix sums
// of c_k / C(N,k)).  Only their signs are used, so all of them are scaled by
// L = lcm_k C(N,k): c_k is multiplied by the integer L / C(N,k) instead of
// being divided (one rounding either way, no FP64 division).
template <int N>
struct BernScale {
  double v[N + 1];
  // C(N,k) and their lcm, exact in integers for the degrees used here
  constexpr BernScale() : v() {
    long long c[N + 1] = {};
    c[0] = 1;
    for (int i = 1; i <= N; ++i) c[i] = c[i - 1] * (N - i + 1) / i;
    long long l = 1;
    for (int i = 0; i <= N; ++i) {
      long long a = l, b = c[i];
      while (b) {
        const long long t = a % b;
        a = b;
        b = t;
      }
      l = l / a * c[i];
    }
    for (int k = 0; k <= N; ++k) v[k] = (double)(l / c[k]);
  }
};
static_assert(BernScale<6>().v[3] == 3.0 && BernScale<6>().v[0] == 60.0, "lcm of C(6,k) is 60");
static_assert(BernScale<3>().v[1] == 1.0 && BernScale<3>().v[3] == 3.0, "lcm of C(3,k) is 3");

// Bernstein coefficients (times L, see BernScale) of f restricted to
// [u, u + wd]: Taylor shift to u, scale by wd^k, then the prefix sums.
template <int N>
__host__ __device__ void bernstein_on(const double f[N + 1], double u, double wd, double b[N + 1]) {
  double c[N + 1];
#pragma unroll
  for (int k = 0; k <= N; ++k) c[k] = f[k];
#pragma unroll
  for (int i = 0; i < N; ++i)
#pragma unroll
    for (int k = N - 1; k >= i; --k) c[k] += u * c[k + 1];
  constexpr BernScale<N> L{};
  double p = 1.0;
#pragma unroll
  for (int k = 0; k <= N; ++k) {
    c[k] *= p * L.v[k];
    p *= wd;
  }
#pragma unroll
  for (int j = 0; j <= N; ++j) b[j] = c[j];
#pragma unroll
  for (int r = 1; r <= N; ++r)
#pragma unroll
    for (int j = N; j >= r; --j) b[j] += b[j - 1];
}

// Root of f in [lo, hi] where f(lo) = flo != 0 and f changes sign (one root
// inside).  Newton steps from a start point (the given guess when it lies
// inside, else the secant point of the bracket), the bracket kept around the
// root; a step that would leave the bracket is replaced by the Illinois point
// (regula falsi with the value at an end that was kept twice in a row
// halved), which still converges superlinearly where Newton would not.
// Stops at an exact zero, a bracket of width 2^-50 or a step below 2^-52 x.
// Newton with this fallback has the shortest tail over a wavefront of the
// variants measured (safeguarded Newton from the midpoint, plain Illinois).
template <int N>
__host__ __device__ double refine(const double f[N + 1], double lo, double hi, double flo, double guess = -1.0) {
  const double tol = 8.881784197001252e-16;
  double fhi = horner<N>(f, hi);
  int side = 0;
  double x = (guess > lo && guess < hi) ? guess : (lo * fhi - hi * flo) / (fhi - flo);
  if (!(x > lo && x < hi)) x = 0.5 * (lo + hi);
  for (int it = 0; it < 100; ++it) {
    double fx = f[N], dfx = 0.0;
#pragma unroll
    for (int k = N - 1; k >= 0; --k) {
      dfx = dfx * x + fx;
      fx = fx * x + f[k];
    }
    if (fx == 0.0) return x;
    if ((fx < 0.0) == (flo < 0.0)) {
      lo = x;
      flo = fx;
      if (side == -1) fhi *= 0.5;
      side = -1;
    } else {
      hi = x;
      fhi = fx;
      if (side == 1) flo *= 0.5;
      side = 1;
    }
    if (hi - lo <= tol) break;
    double xn = (dfx != 0.0) ? x - fx / dfx : -1.0;
    if (!(xn > lo && xn < hi)) xn = (lo * fhi - hi * flo) / (fhi - flo);
    if (!(xn > lo && xn < hi)) xn = 0.5 * (lo + hi);
    if (fabs(xn - x) <= 2.220446049250313e-16 * fmax(fabs(x), 1e-300)) {
      x = xn;
      break;
    }
    x = xn;
  }
  return x;
}

// Budget of one root search: intervals examined (shared by the calls of one
// candidate) and subdivision depth.  A search that runs out of intervals
// stops without a result and is counted in *exh: the caller reports it (its
// contacts may be missing), it is never taken for "no contact".  At the
// depth limit an interval 2^-44 of the search range wide is decided by the
// signs of F at its ends (a root there would be a near-double root).
constexpr int kMaxSearchLevel = 44;
constexpr int kMaxSearchVisits = 4096;

// Earliest valid root of F (degree N, coefficients f) in [lo, hi] by
// depth-first Bernstein subdivision of that interval into the pieces
// lo + (hi - lo) [idx 2^-level, (idx + 1) 2^-level].  Returns 1 with *s_out on
// contact.  *visits counts the intervals examined (shared budget across
// calls); *deg counts degenerate skips, *exh searches that ran out of their
// budget of intervals.  guess (optional) is the start of the refinement of a
// root isolated in an interval that contains it.
//
// With a predicted bracket lo <= blo < bhi <= hi (blo >= 0 to use it): when
// the whole interval neither excludes a root nor isolates one, and the
// Bernstein coefficients of F on [lo, blo] all have one strict sign (no root
// before blo), the traversal continues on [blo, bhi] and then on [bhi, hi]
// instead of the halves of [lo, hi]; *certified is then set.  The roots are
// met in the same left-to-right order, so the result is the same contact.
//
// The search alternates two phases: subdivide until the next interval that
// isolates a root (or the end), then refine that root and test it.  On a
// wavefront, lanes that have isolated a root wait at the end of the first
// phase, so the refinements of all lanes run together once per root instead
// of once per subdivision step of any lane.  The intervals visited and the
// roots computed are those of a plain depth-first traversal.
template <int N>
__host__ __device__ int search_in(const Quad &Q, const double f[N + 1], double lo, double hi, double *s_out,
                                  int *visits, int *deg, int *exh, double guess = -1.0, double blo = -1.0,
                                  double bhi = -1.0, int *certified = nullptr) {
  const int kMaxLevel = kMaxSearchLevel;
  const int kMaxVisits = kMaxSearchVisits;
  // the segment being traversed, and the one after it (when pend_hi > pend_lo)
  double seg_lo = lo, span = hi - lo, pend_lo = 0.0, pend_hi = 0.0;
  bool bracket = blo >= lo && blo < bhi && bhi <= hi;
  int level = 0;
  long long idx = 0;
  bool done = false;
  while (!done) {
    // phase 1: next isolated root (u, v, fu) or a root found directly (root >= 0)
    bool iso = false;
    double u = 0.0, v = 0.0, fu = 0.0, root = -1.0;
    while (!done && !iso) {
      if (++(*visits) > kMaxVisits) {
        (*exh)++;
        return 0;
      }
      const double wd = ldexp(1.0, -level);
      u = seg_lo + span * ((double)idx * wd);
      v = seg_lo + span * ((double)(idx + 1) * wd);
      double b[N + 1];
      bernstein_on<N>(f, u, v - u, b);
      bool pos = true, neg = true;
      int changes = 0, last = 0;
#pragma unroll
      for (int k = 0; k <= N; ++k) {
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
        fu = horner<N>(f, u);
        const double fv = horner<N>(f, v);
        if (changes == 1 && b[0] != 0.0 && b[N] != 0.0 && fu != 0.0 && fv != 0.0 && ((fu < 0.0) != (fv < 0.0))) {
          iso = true;
        } else if (level < kMaxLevel) {
          descend = true;
        } else if (fu == 0.0) {
          root = u;
          iso = true;
        } else if (fv != 0.0 && ((fu < 0.0) != (fv < 0.0))) {
          iso = true;
        }
      }
      if (descend && bracket) {
        // first interval of the search, undecided: try the predicted bracket
        bracket = false;
        bool ok = true;
        if (blo > seg_lo) {
          if (++(*visits) > kMaxVisits) {
            (*exh)++;
            return 0;
          }
          double c[N + 1];
          bernstein_on<N>(f, seg_lo, blo - seg_lo, c);
          bool cp = true, cn = true;
#pragma unroll
          for (int k = 0; k <= N; ++k) {
            cp &= c[k] > 0.0;
            cn &= c[k] < 0.0;
          }
          ok = cp || cn;
        }
        if (ok) {
          if (certified) *certified = 1;
          pend_lo = bhi;
          pend_hi = seg_lo + span;
          seg_lo = blo;
          span = bhi - blo;
          continue;  // level 0, idx 0 of [blo, bhi]
        }
      }
      if (descend) {
        ++level;
        idx <<= 1;
        continue;
      }
      // move past this interval (the traversal resumes there if the root is not valid)
      while (level > 0 && (idx & 1)) { idx >>= 1; --level; }
      if (level > 0) {
        ++idx;
      } else if (pend_hi > pend_lo) {
        seg_lo = pend_lo;
        span = pend_hi - pend_lo;
        pend_lo = pend_hi = 0.0;
        idx = 0;
      } else {
        done = true;
      }
    }
    if (!iso) break;
    // phase 2: refine and test
    if (root < 0.0) root = refine<N>(f, u, v, fu, guess);
    const int in = inside_at(Q, root);
    if (in < 0) (*deg)++;
    if (in == 1) {
      *s_out = root;
      return 1;
    }
  }
  return 0;
}

// Coefficients of F and the two cases settled before any search: F == 0
// identically (degenerate, returns 0) and a vertex within d and inside at
// s = 0 (contact at 0, returns 1).  Returns -1 when a search is needed.
template <int N>
__host__ __device__ inline int prepare(const Quad &Q, double d, double f[N + 1], double *s_out, int *within,
                                       int *deg) {
  poly_coeffs<N>(Q, d, f);
  bool allzero = true;
#pragma unroll
  for (int k = 0; k <= N; ++k) allzero &= (f[k] == 0.0);
  if (allzero) { (*deg)++; return 0; }
  if (N == 6 && f[0] < 0.0 && inside_at(Q, 0.0) == 1) {
    (*within)++;
    *s_out = 0.0;
    return 1;
  }
  return -1;
}

// Earliest valid root of F (degree N) on [0,1].  Returns 1 with *s on contact.
// *deg counts degenerate skips (vanishing normal at a root, or F == 0),
// *exh searches stopped by their budget (search_in).
template <int N>
__host__ __device__ int earliest(const Quad &Q, double d, double *s_out, int *within, int *deg, int *exh) {
  double f[N + 1];
  const int pre = prepare<N>(Q, d, f, s_out, within, deg);
  if (pre >= 0) return pre;
  int visits = 0;
  return search_in<N>(Q, f, 0.0, 1.0, s_out, &visits, deg, exh);
}

// The same earliest valid root, searched with a predicted root `guess` and
// bracket [lo, hi] of [0,1] (search_in: the bracket replaces the halving of
// [0, 1] when that interval is undecided and F has no root before lo; the
// prediction starts the refinement of an isolated root that it lies in).
// The result is the root of earliest() (up to the last bits of the final
// refinement, which starts from a different point).  *certified reports
// whether the bracket was used.
template <int N>
__host__ __device__ int earliest_bracket(const Quad &Q, double d, double lo, double hi, double guess, double *s_out,
                                         int *within, int *deg, int *exh, int *certified) {
  double f[N + 1];
  const int pre = prepare<N>(Q, d, f, s_out, within, deg);
  *certified = 0;
  if (pre >= 0) return pre;
  int visits = 0;
  return search_in<N>(Q, f, 0.0, 1.0, s_out, &visits, deg, exh, guess, lo, hi, certified);
}

// V and dV/dX1 (order p, a, b, c) of a vertex-triangle contact at s.
__host__ __device__ inline void volume_grad(const Quad &Q, double s, double d, double eps, double dt, bool clamped, double *V,
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

// Bernstein coefficients on [0,1] of a degree-4 polynomial c (times 12, the
// lcm of C(4,k)).
__host__ __device__ inline void bern4(const double c[5], double b[5]) {
  constexpr BernScale<4> L{};
#pragma unroll
  for (int k = 0; k <= 4; ++k) b[k] = c[k] * L.v[k];
#pragma unroll
  for (int r = 1; r <= 4; ++r)
#pragma unroll
    for (int j = 4; j >= r; --j) b[j] += b[j - 1];
}

// True if c < -tol on all of [0,1], proved by its Bernstein coefficients
// (times 12: tol is scaled the same way).
__host__ __device__ inline bool below_on01(const double c[5], double tol) {
  double b[5];
  bern4(c, b);
  bool all = true;
#pragma unroll
  for (int k = 0; k <= 4; ++k) all &= b[k] < -12.0 * tol;
  return all;
}

__host__ __device__ inline double norm1(const d3 &a) { return fabs(a.x) + fabs(a.y) + fabs(a.z); }

// False when the closest-point test of the narrow phase fails at every s in
// [0,1], so that no root of F can be a contact.  With the edge vectors u, v,
// w and normal n = u x v of poly_coeffs (all polynomials in s):
// alpha = (w x v).n, beta = (w x u).n, q = |n|^2 (degree 4).  Vertex-triangle
// inside test: alpha >= 0, -beta >= 0, alpha - beta <= q; edge-edge:
// 0 <= alpha <= q and 0 <= beta <= q.  One of these failing with a margin on
// all of [0,1] (Bernstein coefficients) excludes every root.  The margin,
// 1e-10 of a bound on the magnitude of each polynomial on [0,1], is far above
// the rounding of these coefficients and of the test at a root, so the
// decision agrees with the test itself.
__host__ __device__ inline bool may_be_inside(const Quad &Q) {
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
  const d3 n0 = crossp(u0, v0), n1 = crossp(u0, v1) + crossp(u1, v0), n2 = crossp(u1, v1);
  const d3 a0 = crossp(w0, v0), a1 = crossp(w0, v1) + crossp(w1, v0), a2 = crossp(w1, v1);
  const d3 c0 = crossp(w0, u0), c1 = crossp(w0, u1) + crossp(w1, u0), c2 = crossp(w1, u1);
  const double al[5] = {dotp(a0, n0), dotp(a0, n1) + dotp(a1, n0), dotp(a0, n2) + dotp(a1, n1) + dotp(a2, n0),
                        dotp(a1, n2) + dotp(a2, n1), dotp(a2, n2)};
  const double be[5] = {dotp(c0, n0), dotp(c0, n1) + dotp(c1, n0), dotp(c0, n2) + dotp(c1, n1) + dotp(c2, n0),
                        dotp(c1, n2) + dotp(c2, n1), dotp(c2, n2)};
  const double qq[5] = {dotp(n0, n0), 2.0 * dotp(n0, n1), dotp(n1, n1) + 2.0 * dotp(n0, n2), 2.0 * dotp(n1, n2),
                        dotp(n2, n2)};
  const double Nn = norm1(n0) + norm1(n1) + norm1(n2);
  const double Ma = (norm1(w0) + norm1(w1)) * (norm1(v0) + norm1(v1)) * Nn;
  const double Mb = (norm1(w0) + norm1(w1)) * (norm1(u0) + norm1(u1)) * Nn;
  const double Mq = Nn * Nn;
  const double e = 1e-10;
  double t[5];
  if (below_on01(al, e * Ma)) return false;  // alpha < 0 throughout
  if (!Q.ee) {
#pragma unroll
    for (int k = 0; k <= 4; ++k) t[k] = -be[k];
    if (below_on01(t, e * Mb)) return false;  // -beta < 0 throughout
#pragma unroll
    for (int k = 0; k <= 4; ++k) t[k] = (qq[k] - al[k]) + be[k];
    if (below_on01(t, e * (Ma + Mb + Mq))) return false;  // alpha - beta > q throughout
    return true;
  }
  if (below_on01(be, e * Mb)) return false;  // beta < 0 throughout
#pragma unroll
  for (int k = 0; k <= 4; ++k) t[k] = qq[k] - al[k];
  if (below_on01(t, e * (Ma + Mq))) return false;  // alpha > q throughout
#pragma unroll
  for (int k = 0; k <= 4; ++k) t[k] = qq[k] - be[k];
  if (below_on01(t, e * (Mb + Mq))) return false;  // beta > q throughout
  return true;
}

// Screen of one candidate: true if F may have a root in [0,1] or the vertex
// may start within d (the candidate then needs the root search).  Uses the
// Bernstein coefficients on [0,1]: all positive (d > 0) or all of one strict
// sign (d = 0) proves there is neither.
template <int N>
__host__ __device__ inline bool needs_root_search(const Quad &Q, double d) {
  double f[N + 1], b[N + 1];
  poly_coeffs<N>(Q, d, f);
  constexpr BernScale<N> L{};
#pragma unroll
  for (int j = 0; j <= N; ++j) b[j] = f[j] * L.v[j];
#pragma unroll
  for (int r = 1; r <= N; ++r)
#pragma unroll
    for (int j = N; j >= r; --j) b[j] += b[j - 1];
  bool pos = true, neg = true;
#pragma unroll
  for (int k = 0; k <= N; ++k) { pos &= b[k] > 0.0; neg &= b[k] < 0.0; }
  return !(pos || (N == 3 && neg));
}


// ---------------------------------------------------------------------------
// Full gradient of V_k with respect to X0 and X1 of the four vertices, for a
// generic scalar type (double, or Dual for forward-mode derivatives of the
// gradient itself: the Hessian-vector products of the backward pass).
// P(s) = X0 + s D, D = X1 - X0, U_p = D_p / dt, V = 0.5 dt (1 - s) R,
// R = sqrt(eps^2 q + (U_p.n)^2).  dP_j/dX1_j = s, dP_j/dX0_j = 1 - s,
// dU_p/dX1_p = 1/dt = -dU_p/dX0_p; s moves with the positions through
// F(s, X0, X1) = 0: ds/dX1_j = -s F_Pj / F_s, ds/dX0_j = -(1 - s) F_Pj / F_s.
// ---------------------------------------------------------------------------
struct Dual {
  double v, d;
};
__host__ __device__ inline Dual operator+(Dual a, Dual b) { return Dual{a.v + b.v, a.d + b.d}; }
__host__ __device__ inline Dual operator-(Dual a, Dual b) { return Dual{a.v - b.v, a.d - b.d}; }
__host__ __device__ inline Dual operator-(Dual a) { return Dual{-a.v, -a.d}; }
__host__ __device__ inline Dual operator*(Dual a, Dual b) { return Dual{a.v * b.v, a.d * b.v + a.v * b.d}; }
__host__ __device__ inline Dual operator/(Dual a, Dual b) {
  return Dual{a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)};
}
__host__ __device__ inline Dual dsqrt(Dual a) {
  const double r = sqrt(a.v);
  return Dual{r, a.d / (2.0 * r)};
}
__host__ __device__ inline double dsqrt(double a) { return sqrt(a); }
__host__ __device__ inline Dual cst(double x, Dual) { return Dual{x, 0.0}; }
__host__ __device__ inline double cst(double x, double) { return x; }

template <class T>
struct V3 {
  T x, y, z;
};
template <class T>
__host__ __device__ inline V3<T> operator+(V3<T> a, V3<T> b) { return V3<T>{a.x + b.x, a.y + b.y, a.z + b.z}; }
template <class T>
__host__ __device__ inline V3<T> operator-(V3<T> a, V3<T> b) { return V3<T>{a.x - b.x, a.y - b.y, a.z - b.z}; }
template <class T>
__host__ __device__ inline V3<T> scale(T s, V3<T> a) { return V3<T>{s * a.x, s * a.y, s * a.z}; }
template <class T>
__host__ __device__ inline T dot3(V3<T> a, V3<T> b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
template <class T>
__host__ __device__ inline V3<T> cross3(V3<T> a, V3<T> b) {
  return V3<T>{a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}

// X0, X1: (p, a, b, c) with the image shift already applied to X0 and X1.
// Writes V, g0 = dV/dX0 (12), g1 = dV/dX1 (12); dsdx1 (optional, 12) gets
// ds/dX1 of the contact time (zero when clamped at s = 0).
template <class T>
__host__ __device__ void full_grad(const V3<T> X0[4], const V3<T> X1[4], T s, double d, double eps, double dt,
                                   bool clamped, T *V, T g0[12], T g1[12], T *dsdx1) {
  const T one = cst(1.0, s), half = cst(0.5, s), two = cst(2.0, s);
  const T tdt = cst(dt, s), te2 = cst(eps * eps, s), td2 = cst(d * d, s);
  V3<T> D[4], P[4];
  for (int k = 0; k < 4; ++k) {
    D[k] = X1[k] - X0[k];
    P[k] = X0[k] + scale(s, D[k]);
  }
  const V3<T> e1 = P[2] - P[1], e2 = P[3] - P[1], w = P[0] - P[1];
  const V3<T> e1s = D[2] - D[1], e2s = D[3] - D[1], ws = D[0] - D[1];
  const V3<T> n = cross3(e1, e2);
  const T q = dot3(n, n);
  const V3<T> U = scale(one / tdt, D[0]);
  const T un = dot3(U, n);
  const T R = dsqrt(te2 * q + un * un);
  const T k = half * tdt * (one - s);
  *V = k * R;
  const V3<T> m = scale(one / R, scale(te2, n) + scale(un, U));  // dR/dn
  // explicit parts at fixed s (through n for the triangle, through U for p)
  const V3<T> tp = scale(half * (one - s) * un / R, n);
  const V3<T> ta = scale(k, cross3(e1 - e2, m)), tb = scale(k, cross3(e2, m)), tc = scale(k, cross3(m, e1));
  V3<T> G1[4] = {tp, scale(s, ta), scale(s, tb), scale(s, tc)};
  V3<T> G0[4] = {scale(cst(-1.0, s), tp), scale(one - s, ta), scale(one - s, tb), scale(one - s, tc)};
  V3<T> ds1[4];
  const T zero = cst(0.0, s);
  for (int j = 0; j < 4; ++j) ds1[j] = V3<T>{zero, zero, zero};
  if (!clamped) {
    const V3<T> ns = cross3(e1s, e2) + cross3(e1, e2s);
    const T gv = dot3(w, n);
    const T gs = dot3(ws, n) + dot3(w, ns);
    const V3<T> dgp = n, dga = cross3(e1 - e2, w) - n, dgb = cross3(e2, w), dgc = cross3(w, e1);
    T Fs;
    V3<T> FP[4];
    if (d == 0.0) {
      Fs = gs;
      FP[0] = dgp; FP[1] = dga; FP[2] = dgb; FP[3] = dgc;
    } else {
      Fs = two * gv * gs - two * td2 * dot3(n, ns);
      FP[0] = scale(two * gv, dgp);
      FP[1] = scale(two * gv, dga) - scale(td2 * two, cross3(e1 - e2, n));
      FP[2] = scale(two * gv, dgb) - scale(td2 * two, cross3(e2, n));
      FP[3] = scale(two * gv, dgc) - scale(td2 * two, cross3(n, e1));
    }
    const T dVds = half * tdt * (dot3(m, ns) * (one - s) - R);
    for (int j = 0; j < 4; ++j) {
      ds1[j] = scale(cst(-1.0, s) * s / Fs, FP[j]);
      const V3<T> ds0 = scale(cst(-1.0, s) * (one - s) / Fs, FP[j]);
      G1[j] = G1[j] + scale(dVds, ds1[j]);
      G0[j] = G0[j] + scale(dVds, ds0);
    }
  }
  for (int j = 0; j < 4; ++j) {
    g1[3 * j] = G1[j].x; g1[3 * j + 1] = G1[j].y; g1[3 * j + 2] = G1[j].z;
    g0[3 * j] = G0[j].x; g0[3 * j + 1] = G0[j].y; g0[3 * j + 2] = G0[j].z;
    if (dsdx1) { dsdx1[3 * j] = ds1[j].x; dsdx1[3 * j + 1] = ds1[j].y; dsdx1[3 * j + 2] = ds1[j].z; }
  }
}

// Vector-Jacobian product of one vertex-triangle contact for the backward
// pass: with gV = dL/dV_k and w = dL/d(dV_k/dX1) (12), returns
// c0 = dL/dX0 and c1 = dL/dX1 of the four vertices:
//   c = gV grad V_k + d/de [grad V_k](X1 + e w),
// the second term being the Hessian of V_k applied to w (symmetric), by
// forward-mode differentiation of the full gradient.
__host__ __device__ inline void vt_vjp(const V3<double> X0[4], const V3<double> X1[4], double s, double d,
                                       double eps, double dt, bool clamped, double gV, const double w[12],
                                       double c0[12], double c1[12]) {
  double V, g0[12], g1[12], ds1[12];
  full_grad<double>(X0, X1, s, d, eps, dt, clamped, &V, g0, g1, ds1);
  double sdot = 0.0;
  for (int k = 0; k < 12; ++k) sdot += ds1[k] * w[k];
  V3<Dual> X0d[4], X1d[4];
  for (int j = 0; j < 4; ++j) {
    X0d[j] = V3<Dual>{Dual{X0[j].x, 0.0}, Dual{X0[j].y, 0.0}, Dual{X0[j].z, 0.0}};
    X1d[j] = V3<Dual>{Dual{X1[j].x, w[3 * j]}, Dual{X1[j].y, w[3 * j + 1]}, Dual{X1[j].z, w[3 * j + 2]}};
  }
  Dual Vd, g0d[12], g1d[12];
  full_grad<Dual>(X0d, X1d, Dual{s, clamped ? 0.0 : sdot}, d, eps, dt, clamped, &Vd, g0d, g1d, nullptr);
  for (int k = 0; k < 12; ++k) {
    c0[k] = gV * g0[k] + g0d[k].d;
    c1[k] = gV * g1[k] + g1d[k].d;
  }
}

}  // namespace nm
}  // namespace stiv
