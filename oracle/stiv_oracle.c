/*
 * stiv_oracle.c -- plain, slow, FP64 reference of the contact-detection path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header or table with the GPU library.
 *
 * What it computes (Lu, Rahimian & Zorin, "Parallel contact-aware
 * simulations of deformable particles in 3D Stokes flow"):
 *
 *   1. Space-time bounding boxes of every vesicle: the box of all vertex
 *      positions at t_n and t_{n+1}, inflated by d/2 per side (Sec. 3.3.1,
 *      Alg. 2 "getBoundingBox").
 *   2. Candidate vesicle pairs: every pair whose boxes intersect (Alg. 1 and
 *      Sec. 3.3.1 define the set; the Morton grid of Alg. 1 is only a way to
 *      find it, so here it is found by testing all pairs).  Periodic images
 *      are explicit integer shifts sigma of the box length.
 *   3. Primitive candidates inside each vesicle pair: vertex-triangle pairs
 *      in both directions and edge-edge pairs whose space-time boxes
 *      intersect, by testing all primitive pairs (a primitive that misses the
 *      other vesicle's box cannot hit any of its primitives, so those are
 *      dropped first -- an exact reduction).
 *   4. Narrow phase (Eq. 3.1): with linear trajectories P(s) = X0 + s(X1-X0),
 *      s = t/dt in [0,1], the earliest s where the point-plane distance equals
 *      d and the projection lies in the triangle.  Edge-edge uses the same
 *      polynomial with the edge normal.
 *   5. Contact volume of each vertex-triangle contact (Eq. 3.2, App. A) and
 *      its gradient with respect to X1 of the four vertices, including the
 *      dependence of the contact time on X1 (implicit function theorem).
 *   6. Aggregation: one contact volume per vesicle pair, V = sum of V_k, and
 *      the Jacobian rows per (volume, vertex) (Sec. 3.1.2, Sec. 3.3.2).
 *
 * Every floating-point step is IEEE FP64 with no contraction (built with
 * -ffp-contract=off), in the order written here.
 *
 * Root finding uses the derivative chain: the real roots of F' split [0,1]
 * into intervals where F is monotone; a sign change on such an interval holds
 * exactly one root, found by bisection to a width of 2^-50.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Public layout (mirrored by the Python ctypes wrapper).                    */
/* ------------------------------------------------------------------------ */
typedef struct {
  int32_t n_ves, n_vtx, n_scenes, n_topo;
  const int32_t *vtx_off;    /* [n_ves+1] */
  const int32_t *topo_id;    /* [n_ves] */
  const int32_t *scene_off;  /* [n_scenes+1] */
  const double *box_len;     /* [n_scenes][3], 0 = free axis */
  const double *x0, *x1;     /* [3][n_vtx] */
  const int32_t *topo_nv;    /* [n_topo] */
  const int32_t *tri;        /* [sum nt][3] */
  const int32_t *tri_off;    /* [n_topo+1] */
  const int32_t *edge;       /* [sum ne][2] */
  const int32_t *edge_off;   /* [n_topo+1] */
} oracle_scene;

enum { FLAG_ROOT_EDGE = 0, FLAG_INSIDE = 1, FLAG_DOUBLE = 2, FLAG_NEARMISS = 3 };

typedef struct {
  int64_t n_pairs;
  int32_t *pair_ab;     /* [n][2] */
  int32_t *pair_shift;  /* [n][3] */
  double *ves_box;      /* [n_ves][6] lo xyz, hi xyz */
  int64_t n_cand_vt, n_cand_ee;
  int64_t n_cand_list;
  int32_t *cand;        /* [n][4] pair, kind, i, j (only when requested) */
  int64_t n_ct, n_ct_vt, n_ct_ee;
  int32_t *ct_key;      /* [n][4] pair, kind, i, j */
  double *ct_s, *ct_tau, *ct_vol, *ct_grad /*[n][12]*/, *ct_fs_rel;
  int64_t n_vol;
  int32_t *vol_pair;
  double *vol_V;
  int64_t n_jrow;
  int32_t *j_vol, *j_vtx;
  double *j_g;          /* [n][3] */
  int64_t n_initially_within_d, n_degenerate_skipped;
  int64_t n_flag[4];
  double min_margin[4];
  int32_t threads_used;
} oracle_result;

/* ------------------------------------------------------------------------ */
/* Small vector helpers                                                      */
/* ------------------------------------------------------------------------ */
typedef struct { double x, y, z; } v3;
static v3 mk(double x, double y, double z) { v3 r = {x, y, z}; return r; }
static v3 sub(v3 a, v3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
static v3 add(v3 a, v3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
static v3 scl(double s, v3 a) { return mk(s * a.x, s * a.y, s * a.z); }
static double dot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static v3 cross(v3 a, v3 b) {
  return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

/* ------------------------------------------------------------------------ */
/* Polynomials on [0,1]: coefficients c[0..n] in the power basis.            */
/* ------------------------------------------------------------------------ */
static double peval(const double *c, int n, double s) {
  double r = c[n];
  for (int k = n - 1; k >= 0; --k) r = r * s + c[k];
  return r;
}

static int ptrim(const double *c, int n) {
  while (n > 0 && c[n] == 0.0) --n;
  return n;
}

/* Bisection on [lo,hi] where F is monotone and F(lo), F(hi) have opposite
 * signs (both nonzero).  Stops at width 2^-50. */
static double bisect(const double *c, int n, double lo, double hi, double flo) {
  const double tol = 8.881784197001252e-16; /* 2^-50 */
  for (int it = 0; it < 200 && hi - lo > tol; ++it) {
    double mid = 0.5 * (lo + hi);
    double fm = peval(c, n, mid);
    if (fm == 0.0) return mid;
    if ((fm < 0.0) == (flo < 0.0)) { lo = mid; flo = fm; }
    else hi = mid;
  }
  return 0.5 * (lo + hi);
}

/* All roots of F in [0,1] in ascending order (derivative chain).
 * Returns the count; a double root counts only if F is exactly 0 there.
 * `crit_min` (optional) receives the smallest |F| over [0,1]'s critical
 * points and endpoints, used by the general-position diagnostics. */
static int roots01(const double *c_in, int n_in, double *out, double *crit_min) {
  double c[7];
  int n = ptrim(c_in, n_in);
  for (int k = 0; k <= n; ++k) c[k] = c_in[k];
  if (n == 0) {
    if (crit_min) *crit_min = fabs(c[0]);
    return 0;
  }
  double pts[8];
  int np = 0;
  pts[np++] = 0.0;
  if (n >= 2) {
    double dc[6];
    for (int k = 1; k <= n; ++k) dc[k - 1] = (double)k * c[k];
    double crit[6];
    int nc = roots01(dc, n - 1, crit, NULL);
    for (int k = 0; k < nc; ++k)
      if (crit[k] > 0.0 && crit[k] < 1.0) pts[np++] = crit[k];
  }
  pts[np++] = 1.0;
  int nr = 0;
  double fmin = INFINITY;
  double fprev = peval(c, n, pts[0]);
  for (int k = 0; k < np; ++k) {
    double f = (k == 0) ? fprev : peval(c, n, pts[k]);
    if (fabs(f) < fmin) fmin = fabs(f);
    if (f == 0.0) {
      if (nr == 0 || out[nr - 1] != pts[k]) out[nr++] = pts[k];
    } else if (k > 0 && fprev != 0.0 && ((f < 0.0) != (fprev < 0.0))) {
      out[nr++] = bisect(c, n, pts[k - 1], pts[k], fprev);
    }
    fprev = f;
  }
  if (crit_min) *crit_min = fmin;
  return nr;
}

/* ------------------------------------------------------------------------ */
/* Narrow phase (Eq. 3.1).                                                   */
/*                                                                            */
/* Each relative vector r(s) = r0 + s*r1 is linear in s.  For a triangle     */
/* (a,b,c) and vertex p: e1 = Pb-Pa, e2 = Pc-Pa, w = Pp-Pa, n = e1 x e2      */
/* (quadratic), g = w.n (cubic), q = n.n (quartic); F = g^2 - d^2 q.         */
/* For edges (a,b),(c,e): ea = Pb-Pa, eb = Pe-Pc, w = Pc-Pa, m = ea x eb.    */
/* With d = 0 the equation is g = 0 (its square would only double roots).    */
/* ------------------------------------------------------------------------ */
typedef struct {
  v3 X0[4], D[4]; /* shifted X0 and X1-X0 of the four vertices */
  int kind_ee;    /* 0: (p, a, b, c) vertex-triangle; 1: (a, b, c, e) edge-edge */
} prim4;

static v3 pos_at(const prim4 *P, int k, double s) { return add(P->X0[k], scl(s, P->D[k])); }

/* Coefficients of g and q; returns F's coefficients in f[0..6] (degree). */
static int build_poly(const prim4 *P, double d, double g[4], double q[5], double f[7]) {
  v3 u0, u1, v0, v1, w0, w1;
  if (!P->kind_ee) {
    u0 = sub(P->X0[2], P->X0[1]); u1 = sub(P->D[2], P->D[1]);   /* e1 */
    v0 = sub(P->X0[3], P->X0[1]); v1 = sub(P->D[3], P->D[1]);   /* e2 */
    w0 = sub(P->X0[0], P->X0[1]); w1 = sub(P->D[0], P->D[1]);   /* w  */
  } else {
    u0 = sub(P->X0[1], P->X0[0]); u1 = sub(P->D[1], P->D[0]);   /* ea */
    v0 = sub(P->X0[3], P->X0[2]); v1 = sub(P->D[3], P->D[2]);   /* eb */
    w0 = sub(P->X0[2], P->X0[0]); w1 = sub(P->D[2], P->D[0]);   /* w  */
  }
  v3 n0 = cross(u0, v0);
  v3 n1 = add(cross(u0, v1), cross(u1, v0));
  v3 n2 = cross(u1, v1);
  g[0] = dot(w0, n0);
  g[1] = dot(w1, n0) + dot(w0, n1);
  g[2] = dot(w1, n1) + dot(w0, n2);
  g[3] = dot(w1, n2);
  q[0] = dot(n0, n0);
  q[1] = 2.0 * dot(n0, n1);
  q[2] = dot(n1, n1) + 2.0 * dot(n0, n2);
  q[3] = 2.0 * dot(n1, n2);
  q[4] = dot(n2, n2);
  if (d == 0.0) {
    for (int k = 0; k < 4; ++k) f[k] = g[k];
    return 3;
  }
  double d2 = d * d;
  f[0] = g[0] * g[0] - d2 * q[0];
  f[1] = 2.0 * g[0] * g[1] - d2 * q[1];
  f[2] = g[1] * g[1] + 2.0 * g[0] * g[2] - d2 * q[2];
  f[3] = 2.0 * g[0] * g[3] + 2.0 * g[1] * g[2] - d2 * q[3];
  f[4] = g[2] * g[2] + 2.0 * g[1] * g[3] - d2 * q[4];
  f[5] = 2.0 * g[2] * g[3];
  f[6] = g[3] * g[3];
  return 6;
}

/* Inside test at s, division-free.  Returns 1 inside, 0 outside, -1 if the
 * normal vanishes (degenerate).  `margin` gets min(B, C, q-B-C)/q (VT) or
 * min(U, q-U, W, q-W)/q (EE). */
static int inside_at(const prim4 *P, double s, double *margin) {
  v3 A = pos_at(P, 0, s), B = pos_at(P, 1, s), C = pos_at(P, 2, s), E = pos_at(P, 3, s);
  if (!P->kind_ee) {
    /* p = A, triangle (B, C, E) */
    v3 e1 = sub(C, B), e2 = sub(E, B), w = sub(A, B);
    v3 n = cross(e1, e2);
    double q = dot(n, n);
    if (q == 0.0) return -1;
    double bb = dot(cross(w, e2), n);
    double cc = dot(cross(e1, w), n);
    double r = q - bb - cc;
    if (margin) {
      double m = bb < cc ? bb : cc;
      if (r < m) m = r;
      *margin = m / q;
    }
    return (bb >= 0.0 && cc >= 0.0 && bb + cc <= q) ? 1 : 0;
  } else {
    v3 ea = sub(B, A), eb = sub(E, C), w = sub(C, A);
    v3 m = cross(ea, eb);
    double q = dot(m, m);
    if (q == 0.0) return -1;
    double uu = dot(cross(w, eb), m);
    double ww = dot(cross(w, ea), m);
    if (margin) {
      double mm = uu;
      if (q - uu < mm) mm = q - uu;
      if (ww < mm) mm = ww;
      if (q - ww < mm) mm = q - ww;
      *margin = mm / q;
    }
    return (uu >= 0.0 && uu <= q && ww >= 0.0 && ww <= q) ? 1 : 0;
  }
}

typedef struct {
  int64_t within_d, degenerate;
  int64_t flag[4];
  double minm[4];
} diag_t;

static void diag_init(diag_t *g) {
  memset(g, 0, sizeof(*g));
  for (int k = 0; k < 4; ++k) g->minm[k] = INFINITY;
}
static void diag_note(diag_t *g, int k, double m) {
  if (m < g->minm[k]) g->minm[k] = m;
  if (m < 1e-9) g->flag[k]++;
}

/* Earliest valid contact parameter s* in [0,1]; returns 1 on contact. */
static int narrow(const prim4 *P, double d, double *s_out, diag_t *dg) {
  double g[4], q[5], f[7];
  int n = build_poly(P, d, g, q, f);
  int nt = ptrim(f, n);
  if (nt == 0 && f[0] == 0.0) { dg->degenerate++; return 0; }
  double scale = 0.0;
  for (int k = 0; k <= n; ++k) scale += fabs(f[k]);
  /* already within d and inside at s = 0 */
  if (f[0] < 0.0 && d > 0.0) {
    double mg;
    int in = inside_at(P, 0.0, &mg);
    if (in == 1) {
      dg->within_d++;
      *s_out = 0.0;
      return 1;
    }
  }
  double r[8], fmin;
  int nr = roots01(f, n, r, &fmin);
  if (nr == 0) {
    diag_note(dg, FLAG_NEARMISS, fmin / (scale > 0 ? scale : 1.0));
    return 0;
  }
  for (int k = 0; k < nr; ++k) {
    double mg;
    int in = inside_at(P, r[k], &mg);
    if (in < 0) { dg->degenerate++; continue; }
    diag_note(dg, FLAG_INSIDE, fabs(mg));
    /* slope of F at the root relative to its coefficient scale */
    double fs = 0.0;
    for (int j = n; j >= 1; --j) fs = fs * r[k] + (double)j * f[j];
    diag_note(dg, FLAG_DOUBLE, fabs(fs) / (scale > 0 ? scale : 1.0));
    if (in == 1) {
      double edge = r[k] < 1.0 - r[k] ? r[k] : 1.0 - r[k];
      diag_note(dg, FLAG_ROOT_EDGE, edge);
      *s_out = r[k];
      return 1;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Contact volume (Eq. 3.2 with App. A) and its gradient w.r.t. X1.          */
/*                                                                            */
/* V = (dt - tau) sqrt(eps^2 + (U_p . nhat)^2) |t|                            */
/*   = 0.5 dt (1-s) R,   R = sqrt(eps^2 q + (U_p . n)^2),  q = |n|^2,         */
/* everything at s = s*.  The gradient holds X0 fixed; s* moves with X1       */
/* through F(s*, X1) = 0.  Output order: p, a, b, c (3 each).                 */
/* ------------------------------------------------------------------------ */
static void vt_volume(const prim4 *P, double s, double d, double eps, double dt, int clamped,
                      double *V, double grad[12], double *fs_rel) {
  v3 Pp = pos_at(P, 0, s), Pa = pos_at(P, 1, s), Pb = pos_at(P, 2, s), Pc = pos_at(P, 3, s);
  v3 e1 = sub(Pb, Pa), e2 = sub(Pc, Pa), w = sub(Pp, Pa);
  v3 e1s = sub(P->D[2], P->D[1]), e2s = sub(P->D[3], P->D[1]), ws = sub(P->D[0], P->D[1]);
  v3 n = cross(e1, e2);
  double q = dot(n, n);
  v3 U = scl(1.0 / dt, P->D[0]);
  double un = dot(U, n);
  double R = sqrt(eps * eps * q + un * un);
  *V = 0.5 * dt * (1.0 - s) * R;

  v3 m = scl(1.0 / R, add(scl(eps * eps, n), scl(un, U)));   /* dR/dn */
  double k = 0.5 * dt * (1.0 - s);
  /* explicit part at fixed s: dP_j/dX1_j = s */
  v3 gp = scl(0.5 * (1.0 - s) * un / R, n);
  v3 ga = scl(k * s, cross(sub(e1, e2), m));
  v3 gb = scl(k * s, cross(e2, m));
  v3 gc = scl(k * s, cross(m, e1));

  v3 ns = add(cross(e1s, e2), cross(e1, e2s));
  double gval = dot(w, n);
  double gs = dot(ws, n) + dot(w, ns);
  double Fs;
  v3 Fp, Fa, Fb, Fc; /* dF/dP_j */
  v3 dgp = n;
  v3 dga = sub(cross(sub(e1, e2), w), n);
  v3 dgb = cross(e2, w);
  v3 dgc = cross(w, e1);
  if (d == 0.0) {
    Fs = gs;
    Fp = dgp; Fa = dga; Fb = dgb; Fc = dgc;
  } else {
    double d2 = d * d;
    Fs = 2.0 * gval * gs - 2.0 * d2 * dot(n, ns);
    v3 dqa = scl(2.0, cross(sub(e1, e2), n));
    v3 dqb = scl(2.0, cross(e2, n));
    v3 dqc = scl(2.0, cross(n, e1));
    Fp = scl(2.0 * gval, dgp);
    Fa = sub(scl(2.0 * gval, dga), scl(d2, dqa));
    Fb = sub(scl(2.0 * gval, dgb), scl(d2, dqb));
    Fc = sub(scl(2.0 * gval, dgc), scl(d2, dqc));
  }
  double scale = fabs(Fs);
  {
    double a1 = sqrt(dot(Fp, Fp)) + sqrt(dot(Fa, Fa)) + sqrt(dot(Fb, Fb)) + sqrt(dot(Fc, Fc));
    *fs_rel = a1 > 0 ? scale / a1 : INFINITY;
  }
  if (!clamped && Fs != 0.0) {
    double dVds = 0.5 * dt * (-R + (1.0 - s) * dot(m, ns));
    double c = -dVds * s / Fs; /* ds/dX1_j = -s dF/dP_j / F_s */
    gp = add(gp, scl(c, Fp));
    ga = add(ga, scl(c, Fa));
    gb = add(gb, scl(c, Fb));
    gc = add(gc, scl(c, Fc));
  }
  grad[0] = gp.x; grad[1] = gp.y; grad[2] = gp.z;
  grad[3] = ga.x; grad[4] = ga.y; grad[5] = ga.z;
  grad[6] = gb.x; grad[7] = gb.y; grad[8] = gb.z;
  grad[9] = gc.x; grad[10] = gc.y; grad[11] = gc.z;
}

/* ------------------------------------------------------------------------ */
/* Boxes                                                                     */
/* ------------------------------------------------------------------------ */
static double X(const oracle_scene *S, const double *x, int c, int64_t v) { (void)S; return x[(int64_t)c * S->n_vtx + v]; }

static void vertex_box(const oracle_scene *S, int64_t v, double lo[3], double hi[3]) {
  for (int c = 0; c < 3; ++c) {
    double a = X(S, S->x0, c, v), b = X(S, S->x1, c, v);
    lo[c] = a < b ? a : b;
    hi[c] = a < b ? b : a;
  }
}

/* box of a set of global vertices at both times, inflated by h, then shifted */
static void prim_box(const oracle_scene *S, const int64_t *vs, int nv, double h, const double sh[3],
                     double box[6]) {
  double lo[3], hi[3];
  vertex_box(S, vs[0], lo, hi);
  for (int k = 1; k < nv; ++k) {
    double l2[3], h2[3];
    vertex_box(S, vs[k], l2, h2);
    for (int c = 0; c < 3; ++c) {
      if (l2[c] < lo[c]) lo[c] = l2[c];
      if (h2[c] > hi[c]) hi[c] = h2[c];
    }
  }
  for (int c = 0; c < 3; ++c) {
    box[c] = (lo[c] - h) + sh[c];
    box[3 + c] = (hi[c] + h) + sh[c];
  }
}

static int overlap(const double a[6], const double b[6]) {
  for (int c = 0; c < 3; ++c)
    if (!(a[c] <= b[3 + c] && b[c] <= a[3 + c])) return 0;
  return 1;
}

/* ------------------------------------------------------------------------ */
/* Growable arrays for per-pair results                                      */
/* ------------------------------------------------------------------------ */
typedef struct { void *p; int64_t n, cap; size_t el; } vec_t;
static void vpush(vec_t *v, const void *x) {
  if (v->n == v->cap) {
    v->cap = v->cap ? 2 * v->cap : 64;
    v->p = realloc(v->p, (size_t)v->cap * v->el);
  }
  memcpy((char *)v->p + (size_t)v->n * v->el, x, v->el);
  v->n++;
}

typedef struct { int32_t key[4]; double s, vol, grad[12], fs_rel; } contact_t;

typedef struct {
  vec_t cands;     /* int32[4] */
  vec_t contacts;  /* contact_t */
  int64_t n_vt, n_ee;
  diag_t dg;
} pair_out;

/* ------------------------------------------------------------------------ */
/* Pair enumeration (all vesicle pairs of each scene, all image shifts)      */
/* ------------------------------------------------------------------------ */
typedef struct { int32_t a, b, s[3]; } pair_t;

static int pair_cmp(const void *x, const void *y) {
  const pair_t *p = (const pair_t *)x, *q = (const pair_t *)y;
  if (p->a != q->a) return p->a < q->a ? -1 : 1;
  if (p->b != q->b) return p->b < q->b ? -1 : 1;
  for (int c = 0; c < 3; ++c)
    if (p->s[c] != q->s[c]) return p->s[c] < q->s[c] ? -1 : 1;
  return 0;
}

static int lex_positive(const int32_t s[3]) {
  for (int c = 0; c < 3; ++c) {
    if (s[c] > 0) return 1;
    if (s[c] < 0) return 0;
  }
  return 0;
}

static void shift_vec(const double L[3], const int32_t s[3], double sh[3]) {
  for (int c = 0; c < 3; ++c) sh[c] = (double)s[c] * L[c];
}

static void find_pairs(const oracle_scene *S, const double *vbox, vec_t *pairs) {
  for (int sc = 0; sc < S->n_scenes; ++sc) {
    const double *L = S->box_len + 3 * sc;
    for (int a = S->scene_off[sc]; a < S->scene_off[sc + 1]; ++a) {
      for (int b = a; b < S->scene_off[sc + 1]; ++b) {
        const double *A = vbox + 6 * a, *B = vbox + 6 * b;
        int lo[3], hi[3];
        for (int c = 0; c < 3; ++c) {
          if (L[c] > 0.0) {
            lo[c] = (int)floor((A[c] - B[3 + c]) / L[c]) - 1;
            hi[c] = (int)ceil((A[3 + c] - B[c]) / L[c]) + 1;
          } else {
            lo[c] = hi[c] = 0;
          }
        }
        int32_t s[3];
        for (s[0] = lo[0]; s[0] <= hi[0]; ++s[0])
          for (s[1] = lo[1]; s[1] <= hi[1]; ++s[1])
            for (s[2] = lo[2]; s[2] <= hi[2]; ++s[2]) {
              if (a == b && !lex_positive(s)) continue;
              double sh[3], Bs[6];
              shift_vec(L, s, sh);
              for (int c = 0; c < 3; ++c) { Bs[c] = B[c] + sh[c]; Bs[3 + c] = B[3 + c] + sh[c]; }
              if (overlap(A, Bs)) {
                pair_t p = {a, b, {s[0], s[1], s[2]}};
                vpush(pairs, &p);
              }
            }
      }
    }
  }
  qsort(pairs->p, (size_t)pairs->n, sizeof(pair_t), pair_cmp);
}

/* ------------------------------------------------------------------------ */
/* Work inside one vesicle pair                                              */
/* ------------------------------------------------------------------------ */
static void load_prim(const oracle_scene *S, prim4 *P, const int64_t v[4], const double sh[4][3]) {
  for (int k = 0; k < 4; ++k) {
    P->X0[k] = mk(X(S, S->x0, 0, v[k]) + sh[k][0], X(S, S->x0, 1, v[k]) + sh[k][1],
                  X(S, S->x0, 2, v[k]) + sh[k][2]);
    P->D[k] = mk(X(S, S->x1, 0, v[k]) - X(S, S->x0, 0, v[k]), X(S, S->x1, 1, v[k]) - X(S, S->x0, 1, v[k]),
                 X(S, S->x1, 2, v[k]) - X(S, S->x0, 2, v[k]));
  }
}

static void do_pair(const oracle_scene *S, const pair_t *pr, int32_t pidx, const double *vbox, double d,
                    double eps, double dt, int emit, pair_out *out) {
  const double h = 0.5 * d;
  const double zero[3] = {0, 0, 0};
  int sc = 0;
  while (!(pr->a >= S->scene_off[sc] && pr->a < S->scene_off[sc + 1])) ++sc;
  double sh[3];
  shift_vec(S->box_len + 3 * sc, pr->s, sh);
  const int ves[2] = {pr->a, pr->b};
  double vb[2][6];
  for (int c = 0; c < 6; ++c) vb[0][c] = vbox[6 * pr->a + c];
  for (int c = 0; c < 3; ++c) { vb[1][c] = vbox[6 * pr->b + c] + sh[c]; vb[1][3 + c] = vbox[6 * pr->b + 3 + c] + sh[c]; }

  /* filtered primitive lists per side: vertices, triangles, edges (local ids + boxes) */
  int32_t *lv[2], *lt[2], *le[2];
  double *bv[2], *bt[2], *be[2];
  int nv[2], nt[2], ne[2];
  for (int side = 0; side < 2; ++side) {
    int v = ves[side], t = S->topo_id[v];
    int64_t base = S->vtx_off[v];
    const double *shs = side ? sh : zero;
    const double *other = vb[1 - side];
    int NV = S->topo_nv[t];
    int NT = S->tri_off[t + 1] - S->tri_off[t];
    int NE = S->edge_off[t + 1] - S->edge_off[t];
    const int32_t *tri = S->tri + 3 * (int64_t)S->tri_off[t];
    const int32_t *edg = S->edge + 2 * (int64_t)S->edge_off[t];
    lv[side] = malloc(sizeof(int32_t) * NV); bv[side] = malloc(sizeof(double) * 6 * NV);
    lt[side] = malloc(sizeof(int32_t) * NT); bt[side] = malloc(sizeof(double) * 6 * NT);
    le[side] = malloc(sizeof(int32_t) * NE); be[side] = malloc(sizeof(double) * 6 * NE);
    nv[side] = nt[side] = ne[side] = 0;
    for (int i = 0; i < NV; ++i) {
      int64_t g = base + i;
      double bx[6];
      prim_box(S, &g, 1, h, shs, bx);
      if (overlap(bx, other)) { lv[side][nv[side]] = i; memcpy(bv[side] + 6 * nv[side], bx, sizeof bx); nv[side]++; }
    }
    for (int i = 0; i < NT; ++i) {
      int64_t g[3] = {base + tri[3 * i], base + tri[3 * i + 1], base + tri[3 * i + 2]};
      double bx[6];
      prim_box(S, g, 3, h, shs, bx);
      if (overlap(bx, other)) { lt[side][nt[side]] = i; memcpy(bt[side] + 6 * nt[side], bx, sizeof bx); nt[side]++; }
    }
    for (int i = 0; i < NE; ++i) {
      int64_t g[2] = {base + edg[2 * i], base + edg[2 * i + 1]};
      double bx[6];
      prim_box(S, g, 2, h, shs, bx);
      if (overlap(bx, other)) { le[side][ne[side]] = i; memcpy(be[side] + 6 * ne[side], bx, sizeof bx); ne[side]++; }
    }
  }

  /* vertex-triangle, both directions: kind 0 = vertex of a vs triangle of b,
   * kind 1 = vertex of b vs triangle of a.  Keys are sorted (kind, i, j). */
  for (int kind = 0; kind < 2; ++kind) {
    int sv = kind ? 1 : 0, stt = kind ? 0 : 1;
    int vv = ves[sv], vt = ves[stt];
    int64_t basev = S->vtx_off[vv], baset = S->vtx_off[vt];
    const int32_t *tri = S->tri + 3 * (int64_t)S->tri_off[S->topo_id[vt]];
    const double *shv = sv ? sh : zero, *sht = stt ? sh : zero;
    for (int ii = 0; ii < nv[sv]; ++ii) {
      for (int jj = 0; jj < nt[stt]; ++jj) {
        if (!overlap(bv[sv] + 6 * ii, bt[stt] + 6 * jj)) continue;
        int32_t i = lv[sv][ii], j = lt[stt][jj];
        int32_t key[4] = {pidx, kind, i, j};
        out->n_vt++;
        if (emit) vpush(&out->cands, key);
        prim4 P;
        P.kind_ee = 0;
        int64_t g[4] = {basev + i, baset + tri[3 * j], baset + tri[3 * j + 1], baset + tri[3 * j + 2]};
        double shk[4][3];
        for (int c = 0; c < 3; ++c) { shk[0][c] = shv[c]; shk[1][c] = shk[2][c] = shk[3][c] = sht[c]; }
        load_prim(S, &P, g, shk);
        double s;
        if (narrow(&P, d, &s, &out->dg)) {
          contact_t ct;
          memcpy(ct.key, key, sizeof key);
          ct.s = s;
          vt_volume(&P, s, d, eps, dt, s == 0.0, &ct.vol, ct.grad, &ct.fs_rel);
          vpush(&out->contacts, &ct);
        }
      }
    }
  }
  /* edge-edge: kind 2 = edge i of a vs edge j of b */
  {
    int64_t base0 = S->vtx_off[pr->a], base1 = S->vtx_off[pr->b];
    const int32_t *e0 = S->edge + 2 * (int64_t)S->edge_off[S->topo_id[pr->a]];
    const int32_t *e1 = S->edge + 2 * (int64_t)S->edge_off[S->topo_id[pr->b]];
    for (int ii = 0; ii < ne[0]; ++ii) {
      for (int jj = 0; jj < ne[1]; ++jj) {
        if (!overlap(be[0] + 6 * ii, be[1] + 6 * jj)) continue;
        int32_t i = le[0][ii], j = le[1][jj];
        int32_t key[4] = {pidx, 2, i, j};
        out->n_ee++;
        if (emit) vpush(&out->cands, key);
        prim4 P;
        P.kind_ee = 1;
        int64_t g[4] = {base0 + e0[2 * i], base0 + e0[2 * i + 1], base1 + e1[2 * j], base1 + e1[2 * j + 1]};
        double shk[4][3];
        for (int c = 0; c < 3; ++c) { shk[0][c] = shk[1][c] = 0.0; shk[2][c] = shk[3][c] = sh[c]; }
        load_prim(S, &P, g, shk);
        double s;
        if (narrow(&P, d, &s, &out->dg)) {
          contact_t ct;
          memset(&ct, 0, sizeof ct);
          memcpy(ct.key, key, sizeof key);
          ct.s = s;
          vpush(&out->contacts, &ct);
        }
      }
    }
  }
  for (int side = 0; side < 2; ++side) {
    free(lv[side]); free(bv[side]); free(lt[side]); free(bt[side]); free(le[side]); free(be[side]);
  }
}

/* ------------------------------------------------------------------------ */
/* Aggregation helpers                                                       */
/* ------------------------------------------------------------------------ */
typedef struct { int32_t vtx; int32_t order; double g[3]; } jcontrib_t;
static int jc_cmp(const void *x, const void *y) {
  const jcontrib_t *a = (const jcontrib_t *)x, *b = (const jcontrib_t *)y;
  if (a->vtx != b->vtx) return a->vtx < b->vtx ? -1 : 1;
  return a->order < b->order ? -1 : (a->order > b->order);
}

/* ------------------------------------------------------------------------ */
/* Entry point                                                               */
/* ------------------------------------------------------------------------ */
oracle_result *oracle_detect(const oracle_scene *S, double d, double eps, double dt, int emit_candidates,
                             const int64_t *pair_subset, int64_t n_subset, int nthreads) {
  oracle_result *R = calloc(1, sizeof(oracle_result));
  const double h = 0.5 * d;
  /* 1. vesicle boxes */
  R->ves_box = malloc(sizeof(double) * 6 * (size_t)(S->n_ves > 0 ? S->n_ves : 1));
  for (int v = 0; v < S->n_ves; ++v) {
    int64_t n = S->vtx_off[v + 1] - S->vtx_off[v];
    int64_t *ids = malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t k = 0; k < n; ++k) ids[k] = S->vtx_off[v] + k;
    const double z[3] = {0, 0, 0};
    prim_box(S, ids, (int)n, h, z, R->ves_box + 6 * v);
    free(ids);
  }
  /* 2. candidate vesicle pairs */
  vec_t pairs = {NULL, 0, 0, sizeof(pair_t)};
  find_pairs(S, R->ves_box, &pairs);
  R->n_pairs = pairs.n;
  R->pair_ab = malloc(sizeof(int32_t) * 2 * (size_t)(pairs.n + 1));
  R->pair_shift = malloc(sizeof(int32_t) * 3 * (size_t)(pairs.n + 1));
  const pair_t *P = (const pair_t *)pairs.p;
  for (int64_t k = 0; k < pairs.n; ++k) {
    R->pair_ab[2 * k] = P[k].a; R->pair_ab[2 * k + 1] = P[k].b;
    for (int c = 0; c < 3; ++c) R->pair_shift[3 * k + c] = P[k].s[c];
  }
  /* 3-5. per pair, in parallel, deterministic output order */
  int64_t nwork = pair_subset ? n_subset : pairs.n;
  pair_out *po = calloc((size_t)(nwork > 0 ? nwork : 1), sizeof(pair_out));
  int used = 1;
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel
  {
#pragma omp single
    used = omp_get_num_threads();
  }
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int64_t w = 0; w < nwork; ++w) {
    int64_t k = pair_subset ? pair_subset[w] : w;
    po[w].cands.el = sizeof(int32_t) * 4;
    po[w].contacts.el = sizeof(contact_t);
    diag_init(&po[w].dg);
    if (k < 0 || k >= pairs.n) continue;
    do_pair(S, &P[k], (int32_t)k, R->ves_box, d, eps, dt, emit_candidates, &po[w]);
  }
  R->threads_used = used;
  /* gather */
  int64_t ncand = 0, nct = 0;
  for (int k = 0; k < 4; ++k) R->min_margin[k] = INFINITY;
  for (int64_t w = 0; w < nwork; ++w) {
    R->n_cand_vt += po[w].n_vt;
    R->n_cand_ee += po[w].n_ee;
    ncand += po[w].cands.n;
    nct += po[w].contacts.n;
    R->n_initially_within_d += po[w].dg.within_d;
    R->n_degenerate_skipped += po[w].dg.degenerate;
    for (int k = 0; k < 4; ++k) {
      R->n_flag[k] += po[w].dg.flag[k];
      if (po[w].dg.minm[k] < R->min_margin[k]) R->min_margin[k] = po[w].dg.minm[k];
    }
  }
  R->n_cand_list = ncand;
  R->cand = malloc(sizeof(int32_t) * 4 * (size_t)(ncand + 1));
  R->n_ct = nct;
  R->ct_key = malloc(sizeof(int32_t) * 4 * (size_t)(nct + 1));
  R->ct_s = malloc(sizeof(double) * (size_t)(nct + 1));
  R->ct_tau = malloc(sizeof(double) * (size_t)(nct + 1));
  R->ct_vol = malloc(sizeof(double) * (size_t)(nct + 1));
  R->ct_fs_rel = malloc(sizeof(double) * (size_t)(nct + 1));
  R->ct_grad = malloc(sizeof(double) * 12 * (size_t)(nct + 1));
  int64_t ic = 0, it = 0;
  for (int64_t w = 0; w < nwork; ++w) {
    memcpy(R->cand + 4 * ic, po[w].cands.p, sizeof(int32_t) * 4 * (size_t)po[w].cands.n);
    ic += po[w].cands.n;
    const contact_t *c = (const contact_t *)po[w].contacts.p;
    for (int64_t k = 0; k < po[w].contacts.n; ++k, ++it) {
      memcpy(R->ct_key + 4 * it, c[k].key, sizeof(int32_t) * 4);
      R->ct_s[it] = c[k].s;
      R->ct_tau[it] = c[k].s * dt;
      R->ct_vol[it] = c[k].vol;
      R->ct_fs_rel[it] = c[k].fs_rel;
      memcpy(R->ct_grad + 12 * it, c[k].grad, sizeof(double) * 12);
      if (c[k].key[1] == 2) R->n_ct_ee++; else R->n_ct_vt++;
    }
  }
  /* 6. aggregation: contacts are already in canonical (pair, kind, i, j) order
   * (pairs ascend in the work list when no subset is given; subsets are
   * processed in the given order, which callers keep ascending). */
  R->vol_pair = malloc(sizeof(int32_t) * (size_t)(nct + 1));
  R->vol_V = malloc(sizeof(double) * (size_t)(nct + 1));
  R->j_vol = malloc(sizeof(int32_t) * 4 * (size_t)(nct + 1));
  R->j_vtx = malloc(sizeof(int32_t) * 4 * (size_t)(nct + 1));
  R->j_g = malloc(sizeof(double) * 12 * (size_t)(nct + 1));
  jcontrib_t *jc = malloc(sizeof(jcontrib_t) * 4 * (size_t)(nct + 1));
  int64_t k0 = 0;
  while (k0 < nct) {
    int32_t pidx = R->ct_key[4 * k0];
    int64_t k1 = k0;
    while (k1 < nct && R->ct_key[4 * k1] == pidx) ++k1;
    int64_t nvt = 0;
    double V = 0.0;
    int njc = 0;
    const pair_t *pr = &P[pidx];
    const int32_t *tri_a = S->tri + 3 * (int64_t)S->tri_off[S->topo_id[pr->a]];
    const int32_t *tri_b = S->tri + 3 * (int64_t)S->tri_off[S->topo_id[pr->b]];
    for (int64_t k = k0; k < k1; ++k) {
      int kind = R->ct_key[4 * k + 1];
      if (kind == 2) continue;
      nvt++;
      V += R->ct_vol[k];
      int vv = kind ? pr->b : pr->a, vt = kind ? pr->a : pr->b;
      const int32_t *tri = kind ? tri_a : tri_b;
      int32_t i = R->ct_key[4 * k + 2], j = R->ct_key[4 * k + 3];
      int32_t gid[4] = {S->vtx_off[vv] + i, S->vtx_off[vt] + tri[3 * j], S->vtx_off[vt] + tri[3 * j + 1],
                        S->vtx_off[vt] + tri[3 * j + 2]};
      for (int r = 0; r < 4; ++r) {
        jc[njc].vtx = gid[r];
        jc[njc].order = njc;
        memcpy(jc[njc].g, R->ct_grad + 12 * k + 3 * r, sizeof(double) * 3);
        njc++;
      }
    }
    if (nvt > 0) {
      int64_t vid = R->n_vol++;
      R->vol_pair[vid] = pidx;
      R->vol_V[vid] = V;
      qsort(jc, (size_t)njc, sizeof(jcontrib_t), jc_cmp);
      int a = 0;
      while (a < njc) {
        int b = a;
        double g[3] = {0, 0, 0};
        while (b < njc && jc[b].vtx == jc[a].vtx) {
          for (int c = 0; c < 3; ++c) g[c] += jc[b].g[c];
          ++b;
        }
        int64_t r = R->n_jrow++;
        R->j_vol[r] = (int32_t)vid;
        R->j_vtx[r] = jc[a].vtx;
        memcpy(R->j_g + 3 * r, g, sizeof g);
        a = b;
      }
    }
    k0 = k1;
  }
  free(jc);
  for (int64_t w = 0; w < nwork; ++w) { free(po[w].cands.p); free(po[w].contacts.p); }
  free(po);
  free(pairs.p);
  return R;
}

void oracle_free(oracle_result *R) {
  if (!R) return;
  free(R->pair_ab); free(R->pair_shift); free(R->ves_box); free(R->cand);
  free(R->ct_key); free(R->ct_s); free(R->ct_tau); free(R->ct_vol); free(R->ct_grad); free(R->ct_fs_rel);
  free(R->vol_pair); free(R->vol_V); free(R->j_vol); free(R->j_vtx); free(R->j_g);
  free(R);
}

/* ------------------------------------------------------------------------ */
/* Single-primitive entry points for the unit pins.                          */
/* x0, x1: [4][3] positions of (p, a, b, c) for VT or (a, b, c, e) for EE.   */
/* ------------------------------------------------------------------------ */
static void prim_from(prim4 *P, const double *x0, const double *x1, int ee) {
  P->kind_ee = ee;
  for (int k = 0; k < 4; ++k) {
    P->X0[k] = mk(x0[3 * k], x0[3 * k + 1], x0[3 * k + 2]);
    P->D[k] = mk(x1[3 * k] - x0[3 * k], x1[3 * k + 1] - x0[3 * k + 1], x1[3 * k + 2] - x0[3 * k + 2]);
  }
}

int oracle_narrow(const double *x0, const double *x1, int ee, double d, double *s_out, int64_t *within_d) {
  prim4 P;
  prim_from(&P, x0, x1, ee);
  diag_t dg;
  diag_init(&dg);
  int hit = narrow(&P, d, s_out, &dg);
  if (within_d) *within_d = dg.within_d;
  return hit;
}

void oracle_vt_volume(const double *x0, const double *x1, double s, double d, double eps, double dt,
                      double *V, double *grad) {
  prim4 P;
  prim_from(&P, x0, x1, 0);
  double fs;
  vt_volume(&P, s, d, eps, dt, s == 0.0, V, grad, &fs);
}

void oracle_poly(const double *x0, const double *x1, int ee, double d, double *f) {
  prim4 P;
  prim_from(&P, x0, x1, ee);
  double g[4], q[5];
  for (int k = 0; k < 7; ++k) f[k] = 0.0;
  build_poly(&P, d, g, q, f);
}

int oracle_roots01(const double *c, int n, double *out) { return roots01(c, n, out, NULL); }

/* ------------------------------------------------------------------------ */
/* Sort and scatter of check points (Alg. 1 step 2, Table 3).                */
/* A stable sort of the Morton keys; equal keys keep ascending global check  */
/* point index.  perm[k] = global index of the k-th sorted check point; the  */
/* per-point values are then gathered through perm ("scattered" rows).       */
/* ------------------------------------------------------------------------ */
void oracle_sort_scatter(int64_t n, const uint64_t *keys, const int64_t *idx, uint64_t *keys_out,
                         int64_t *perm_out) {
  /* insertion sort: O(n^2), stable, obviously correct; used on tiny inputs */
  for (int64_t k = 0; k < n; ++k) { keys_out[k] = keys[k]; perm_out[k] = idx[k]; }
  for (int64_t k = 1; k < n; ++k) {
    uint64_t kk = keys_out[k];
    int64_t pk = perm_out[k];
    int64_t j = k - 1;
    while (j >= 0 && keys_out[j] > kk) {
      keys_out[j + 1] = keys_out[j];
      perm_out[j + 1] = perm_out[j];
      --j;
    }
    keys_out[j + 1] = kk;
    perm_out[j + 1] = pk;
  }
}

/* ------------------------------------------------------------------------ */
/* Backward pass of one vertex-triangle contact by the complex-step method.  */
/*                                                                            */
/* V_k and its gradient with respect to X0 and X1 of (p, a, b, c) are        */
/* written once in complex arithmetic.  Evaluating them at X1 + i h w (h =   */
/* 1e-30), with the contact time s moved to the complex root of F by Newton  */
/* steps, gives in the imaginary parts h times the directional derivative    */
/* of the gradient along w, i.e. the Hessian of V_k applied to w, to machine  */
/* precision (no subtractive cancellation).  The vector-Jacobian product of   */
/* the pair (V_k, dV_k/dX1) with cotangents (gV, w) is then                   */
/*   dL/dX = gV grad V_k + Im(grad V_k(X1 + i h w)) / h.                      */
/* ------------------------------------------------------------------------ */
typedef struct { double complex x, y, z; } c3;
static c3 cmk(double complex x, double complex y, double complex z) { c3 r = {x, y, z}; return r; }
static c3 cadd(c3 a, c3 b) { return cmk(a.x + b.x, a.y + b.y, a.z + b.z); }
static c3 csub(c3 a, c3 b) { return cmk(a.x - b.x, a.y - b.y, a.z - b.z); }
static c3 cscl(double complex s, c3 a) { return cmk(s * a.x, s * a.y, s * a.z); }
static double complex cdot(c3 a, c3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static c3 ccross(c3 a, c3 b) {
  return cmk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}

/* F(s) and dF/ds for complex positions (vertex p, triangle a, b, c) */
static void cF(const c3 X0[4], const c3 D[4], double complex s, double d, double complex *F, double complex *Fs) {
  c3 P[4];
  for (int k = 0; k < 4; ++k) P[k] = cadd(X0[k], cscl(s, D[k]));
  c3 e1 = csub(P[2], P[1]), e2 = csub(P[3], P[1]), w = csub(P[0], P[1]);
  c3 e1s = csub(D[2], D[1]), e2s = csub(D[3], D[1]), ws = csub(D[0], D[1]);
  c3 n = ccross(e1, e2), ns = cadd(ccross(e1s, e2), ccross(e1, e2s));
  double complex g = cdot(w, n), gs = cdot(ws, n) + cdot(w, ns);
  if (d == 0.0) { *F = g; *Fs = gs; return; }
  *F = g * g - d * d * cdot(n, n);
  *Fs = 2.0 * g * gs - 2.0 * d * d * cdot(n, ns);
}

/* V, dV/dX0 (g0) and dV/dX1 (g1) in complex arithmetic at contact time s */
static void cgrad(const c3 X0[4], const c3 X1[4], double complex s, double d, double eps, double dt, int clamped,
                  double complex *V, double complex g0[12], double complex g1[12]) {
  c3 D[4], P[4];
  for (int k = 0; k < 4; ++k) { D[k] = csub(X1[k], X0[k]); P[k] = cadd(X0[k], cscl(s, D[k])); }
  c3 e1 = csub(P[2], P[1]), e2 = csub(P[3], P[1]), w = csub(P[0], P[1]);
  c3 e1s = csub(D[2], D[1]), e2s = csub(D[3], D[1]), ws = csub(D[0], D[1]);
  c3 n = ccross(e1, e2);
  double complex q = cdot(n, n);
  c3 U = cscl(1.0 / dt, D[0]);
  double complex un = cdot(U, n);
  double complex R = csqrt(eps * eps * q + un * un);
  *V = 0.5 * dt * (1.0 - s) * R;
  c3 m = cscl(1.0 / R, cadd(cscl(eps * eps, n), cscl(un, U)));
  double complex k = 0.5 * dt * (1.0 - s);
  /* through U for p (dU/dX1 = 1/dt, dU/dX0 = -1/dt), through n for the triangle */
  c3 tp = cscl(0.5 * (1.0 - s) * un / R, n);
  c3 ta = cscl(k, ccross(csub(e1, e2), m)), tb = cscl(k, ccross(e2, m)), tc = cscl(k, ccross(m, e1));
  c3 G1[4] = {tp, cscl(s, ta), cscl(s, tb), cscl(s, tc)};
  c3 G0[4] = {cscl(-1.0, tp), cscl(1.0 - s, ta), cscl(1.0 - s, tb), cscl(1.0 - s, tc)};
  if (!clamped) {
    c3 ns = cadd(ccross(e1s, e2), ccross(e1, e2s));
    double complex gv = cdot(w, n), gs = cdot(ws, n) + cdot(w, ns);
    c3 dg[4] = {n, csub(ccross(csub(e1, e2), w), n), ccross(e2, w), ccross(w, e1)};
    c3 FP[4];
    double complex Fs;
    if (d == 0.0) {
      Fs = gs;
      for (int j = 0; j < 4; ++j) FP[j] = dg[j];
    } else {
      Fs = 2.0 * gv * gs - 2.0 * d * d * cdot(n, ns);
      c3 dq[4] = {cmk(0, 0, 0), cscl(2.0, ccross(csub(e1, e2), n)), cscl(2.0, ccross(e2, n)), cscl(2.0, ccross(n, e1))};
      for (int j = 0; j < 4; ++j) FP[j] = csub(cscl(2.0 * gv, dg[j]), cscl(d * d, dq[j]));
    }
    double complex dVds = 0.5 * dt * (-R + (1.0 - s) * cdot(m, ns));
    for (int j = 0; j < 4; ++j) {
      G1[j] = cadd(G1[j], cscl(-dVds * s / Fs, FP[j]));
      G0[j] = cadd(G0[j], cscl(-dVds * (1.0 - s) / Fs, FP[j]));
    }
  }
  for (int j = 0; j < 4; ++j) {
    g1[3 * j] = G1[j].x; g1[3 * j + 1] = G1[j].y; g1[3 * j + 2] = G1[j].z;
    g0[3 * j] = G0[j].x; g0[3 * j + 1] = G0[j].y; g0[3 * j + 2] = G0[j].z;
  }
}

/* Real V and gradients with respect to X0 and X1 (12 each, order p, a, b, c). */
void oracle_vt_grad_full(const double *x0, const double *x1, double s, double d, double eps, double dt, double *V,
                         double *g0, double *g1) {
  c3 X0[4], X1[4];
  for (int k = 0; k < 4; ++k) {
    X0[k] = cmk(x0[3 * k], x0[3 * k + 1], x0[3 * k + 2]);
    X1[k] = cmk(x1[3 * k], x1[3 * k + 1], x1[3 * k + 2]);
  }
  double complex Vc, a[12], b[12];
  cgrad(X0, X1, s, d, eps, dt, s == 0.0, &Vc, a, b);
  *V = creal(Vc);
  for (int k = 0; k < 12; ++k) { g0[k] = creal(a[k]); g1[k] = creal(b[k]); }
}

/* dL/dX0, dL/dX1 of one contact for cotangents gV (of V_k) and w (of dV_k/dX1). */
void oracle_vt_backward(const double *x0, const double *x1, double s, double d, double eps, double dt, double gV,
                        const double *w, double *gx0, double *gx1) {
  const double h = 1e-30;
  c3 X0[4], X1[4], D[4];
  for (int k = 0; k < 4; ++k) {
    X0[k] = cmk(x0[3 * k], x0[3 * k + 1], x0[3 * k + 2]);
    X1[k] = cmk(x1[3 * k] + I * h * w[3 * k], x1[3 * k + 1] + I * h * w[3 * k + 1], x1[3 * k + 2] + I * h * w[3 * k + 2]);
    D[k] = csub(X1[k], X0[k]);
  }
  double complex sc = s;
  if (s != 0.0) {
    for (int it = 0; it < 8; ++it) { /* Newton to the complex root near the real one */
      double complex F, Fs;
      cF(X0, D, sc, d, &F, &Fs);
      sc -= F / Fs;
    }
  }
  double complex Vc, a[12], b[12];
  cgrad(X0, X1, sc, d, eps, dt, s == 0.0, &Vc, a, b);
  for (int k = 0; k < 12; ++k) {
    gx0[k] = gV * creal(a[k]) + cimag(a[k]) / h;
    gx1[k] = gV * creal(b[k]) + cimag(b[k]) / h;
  }
}

/* ------------------------------------------------------------------------ */
/* Training samples for the learned contact-time bracket.                    */
/* For each candidate key (pair, kind, i, j): 18 features -- the other three */
/* vertices relative to vertex a (vertex-triangle: b-a, c-a, p-a; edge-edge: */
/* b-a, c-a, e-a) at t_n then at t_{n+1}, divided by the mean edge length of  */
/* the primitives at t_n -- and the label: the first root of F in [0,1]      */
/* (-1 if none).  hard[k] = 1 unless the                                     */
/* Bernstein coefficients of F on [0,1] are all positive (d > 0) or all of   */
/* one strict sign (d = 0), which excludes any root without a search.        */
/* ------------------------------------------------------------------------ */
static double binom(int n, int k) {
  double r = 1.0;
  for (int i = 1; i <= k; ++i) r = r * (double)(n - k + i) / (double)i;
  return r;
}

void oracle_toi_samples(const oracle_scene *S, double d, const int32_t *keys, int64_t n, const int32_t *pair_ab,
                        const int32_t *pair_shift, float *feat, double *root, int8_t *hard, int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static)
#endif
  for (int64_t k = 0; k < n; ++k) {
    const int32_t *key = keys + 4 * k;
    int p = key[0], kind = key[1], i = key[2], j = key[3];
    int a = pair_ab[2 * p], b = pair_ab[2 * p + 1];
    int sc = 0;
    while (!(a >= S->scene_off[sc] && a < S->scene_off[sc + 1])) ++sc;
    double sh[3];
    for (int c = 0; c < 3; ++c) sh[c] = (double)pair_shift[3 * p + c] * S->box_len[3 * sc + c];
    const double zero[3] = {0, 0, 0};
    int64_t g[4];
    const double *shk[4];
    prim4 P;
    if (kind == 2) {
      const int32_t *e0 = S->edge + 2 * ((int64_t)S->edge_off[S->topo_id[a]] + i);
      const int32_t *e1 = S->edge + 2 * ((int64_t)S->edge_off[S->topo_id[b]] + j);
      g[0] = S->vtx_off[a] + e0[0]; g[1] = S->vtx_off[a] + e0[1];
      g[2] = S->vtx_off[b] + e1[0]; g[3] = S->vtx_off[b] + e1[1];
      shk[0] = shk[1] = zero; shk[2] = shk[3] = sh;
      P.kind_ee = 1;
    } else {
      int vv = kind ? b : a, vt = kind ? a : b;
      const int32_t *tri = S->tri + 3 * ((int64_t)S->tri_off[S->topo_id[vt]] + j);
      g[0] = S->vtx_off[vv] + i;
      for (int r = 0; r < 3; ++r) g[1 + r] = S->vtx_off[vt] + tri[r];
      shk[0] = kind ? sh : zero;
      shk[1] = shk[2] = shk[3] = kind ? zero : sh;
      P.kind_ee = 0;
    }
    double shv[4][3];
    for (int r = 0; r < 4; ++r)
      for (int c = 0; c < 3; ++c) shv[r][c] = shk[r][c];
    load_prim(S, &P, g, shv);
    /* features: anchor = vertex a of the primitive pair (index 1 for VT, 0 for EE) */
    int anc = P.kind_ee ? 0 : 1;
    int others[3];
    if (P.kind_ee) { others[0] = 1; others[1] = 2; others[2] = 3; }
    else { others[0] = 2; others[1] = 3; others[2] = 0; }
    double ell;
    if (P.kind_ee) {
      ell = 0.5 * (sqrt(dot(sub(P.X0[1], P.X0[0]), sub(P.X0[1], P.X0[0]))) +
                   sqrt(dot(sub(P.X0[3], P.X0[2]), sub(P.X0[3], P.X0[2]))));
    } else {
      ell = (sqrt(dot(sub(P.X0[2], P.X0[1]), sub(P.X0[2], P.X0[1]))) +
             sqrt(dot(sub(P.X0[3], P.X0[1]), sub(P.X0[3], P.X0[1]))) +
             sqrt(dot(sub(P.X0[3], P.X0[2]), sub(P.X0[3], P.X0[2])))) / 3.0;
    }
    if (!(ell > 0)) ell = 1.0;
    for (int t = 0; t < 2; ++t)
      for (int r = 0; r < 3; ++r) {
        v3 A = t ? add(P.X0[anc], P.D[anc]) : P.X0[anc];
        v3 B = t ? add(P.X0[others[r]], P.D[others[r]]) : P.X0[others[r]];
        v3 rel = sub(B, A);
        feat[18 * k + 9 * t + 3 * r + 0] = (float)(rel.x / ell);
        feat[18 * k + 9 * t + 3 * r + 1] = (float)(rel.y / ell);
        feat[18 * k + 9 * t + 3 * r + 2] = (float)(rel.z / ell);
      }
    double gco[4], q[5], f[7];
    int deg = build_poly(&P, d, gco, q, f);
    {
      /* Bernstein coefficients on [0,1]: b_j = sum_{i<=j} C(j,i)/C(deg,i) f_i */
      int pos = 1, neg = 1;
      for (int j = 0; j <= deg; ++j) {
        double bj = 0.0;
        for (int i = 0; i <= j; ++i) bj += binom(j, i) / binom(deg, i) * f[i];
        pos &= bj > 0.0;
        neg &= bj < 0.0;
      }
      hard[k] = (int8_t)!(pos || (d == 0.0 && neg));
    }
    double r[8];
    int nr = roots01(f, deg, r, NULL);
    root[k] = nr > 0 ? r[0] : -1.0;
  }
}
