// Host build of the root search of the narrow phase (narrow_math.h is
// __host__ __device__): the search with a predicted bracket and start point
// (the learned contact-time bracket) must find the same earliest contact as
// the plain search of Eq. 3.1, whatever the prediction: near the root, far
// from it, before it, after it (then F has a root before the bracket and
// the bracket is not used), touching 0 or 1.
#include <cmath>
#include <cstdio>
#include <random>

#include "narrow_math.h"

using namespace stiv::nm;

static d3 rnd3(std::mt19937_64 &g, double a) {
  std::uniform_real_distribution<double> u(-a, a);
  return mk(u(g), u(g), u(g));
}

// A vertex (or an edge) passing through a triangle's plane (or another
// edge) during the step, plus a random drift of every vertex.
static Quad random_quad(std::mt19937_64 &g, bool ee) {
  std::uniform_real_distribution<double> u01(0.0, 1.0);
  Quad Q;
  Q.ee = ee;
  const d3 a = rnd3(g, 1.0), b = a + rnd3(g, 1.0), c = a + rnd3(g, 1.0);
  const d3 n = crossp(b - a, c - a);
  const double nn = std::sqrt(dotp(n, n));
  const d3 nh = (1.0 / nn) * n;
  const double h = 0.05 + 0.5 * u01(g);
  if (!ee) {
    const double w1 = u01(g), w2 = (1.0 - w1) * u01(g);
    const d3 p = a + w1 * (b - a) + w2 * (c - a) + (u01(g) < 0.3 ? rnd3(g, 0.3) : mk(0, 0, 0));
    Q.X0[0] = p + h * nh;
    Q.D[0] = (-(h + 0.5 * h * u01(g))) * nh + rnd3(g, 0.05);
    Q.X0[1] = a; Q.X0[2] = b; Q.X0[3] = c;
  } else {
    const d3 m = a + 0.5 * (b - a);
    const d3 e = crossp(b - a, nh);
    Q.X0[0] = a; Q.X0[1] = b;
    Q.X0[2] = m + h * nh - 0.6 * e + rnd3(g, 0.1);
    Q.X0[3] = m + h * nh + 0.6 * e + rnd3(g, 0.1);
    const d3 dv = (-(h + 0.5 * h * u01(g))) * nh;
    Q.D[2] = dv + rnd3(g, 0.05);
    Q.D[3] = dv + rnd3(g, 0.05);
  }
  for (int k = 0; k < 4; ++k)
    if (!(k == 0 && !ee) && !(k >= 2 && ee)) Q.D[k] = rnd3(g, 0.05);
  return Q;
}

template <int N>
static int check(std::mt19937_64 &g, int n, double d, int *n_hit, int *n_used) {
  std::uniform_real_distribution<double> u01(0.0, 1.0);
  int fails = 0;
  for (int t = 0; t < n; ++t) {
    const Quad Q = random_quad(g, t % 3 == 2);
    int within = 0, deg = 0, exh = 0;
    double s = -1.0;
    const int hit = earliest<N>(Q, d, &s, &within, &deg, &exh);
    *n_hit += hit;
    for (int k = 0; k < 7; ++k) {
      double lo, hi, guess;
      const double r = hit ? s : u01(g);
      switch (k) {
        case 0: lo = r - 0.05; hi = r + 0.05; guess = r; break;            // good prediction
        case 1: lo = r - 0.2; hi = r + 0.01; guess = r - 0.1; break;       // skewed
        case 2: lo = u01(g); hi = lo + 0.3 * u01(g) + 1e-3; guess = 0.5 * (lo + hi); break;  // random
        case 3: lo = r + 0.1; hi = r + 0.3; guess = r + 0.2; break;        // after the root
        case 4: lo = 0.0; hi = r + 0.1; guess = r; break;                  // touching 0
        case 5: lo = r - 0.1; hi = 1.0; guess = -1.0; break;               // touching 1, no start point
        default: lo = r - 0.3; hi = r - 0.1; guess = r - 0.2; break;      // before the root
      }
      lo = lo < 0.0 ? 0.0 : lo;
      hi = hi > 1.0 ? 1.0 : hi;
      if (!(lo < hi)) continue;
      int w2 = 0, deg2 = 0, exh2 = 0, cert = 0;
      double s2 = -1.0;
      const int hit2 = earliest_bracket<N>(Q, d, lo, hi, guess, &s2, &w2, &deg2, &exh2, &cert);
      *n_used += cert;
      const bool same = hit2 == hit && exh2 == exh && w2 == within && (!hit || std::fabs(s2 - s) <= 1e-12);
      if (!same) {
        if (fails < 10)
          std::printf("mismatch N=%d t=%d k=%d: plain hit=%d s=%.17g exh=%d, bracket [%.6f, %.6f] hit=%d s=%.17g exh=%d\n",
                      N, t, k, hit, s, exh, lo, hi, hit2, s2, exh2);
        ++fails;
      }
    }
  }
  return fails;
}

int main() {
  std::mt19937_64 g(12345);
  int fails = 0, hits6 = 0, used6 = 0, hits3 = 0, used3 = 0;
  fails += check<6>(g, 20000, 0.05, &hits6, &used6);
  fails += check<3>(g, 20000, 0.0, &hits3, &used3);
  std::printf("d>0: %d hits, bracket used %d times; d=0: %d hits, bracket used %d times\n", hits6, used6, hits3, used3);
  std::printf(fails ? "FAIL %d\n" : "OK\n", fails);
  return fails ? 1 : 0;
}
