// Host build of the root search of the narrow phase (narrow_math.h is
// __host__ __device__): drives search_in to its budget of intervals and
// checks that this is counted as exhausted, never as "no contact".
#include <cmath>
#include <cstdio>

#include "narrow_math.h"

using namespace stiv::nm;

// A vertex-triangle quad: the vertex moves from z = 0.5 down through the
// plane of the unit right triangle, at (px, px) (inside for px = 0.2,
// outside for px = 2).  search_in takes its coefficients as given, so a
// test polynomial can be searched with this quad's inside test.
static Quad unit_quad(double px) {
  Quad Q;
  Q.ee = false;
  Q.X0[0] = mk(px, px, 0.5);
  Q.X0[1] = mk(0.0, 0.0, 0.0);
  Q.X0[2] = mk(1.0, 0.0, 0.0);
  Q.X0[3] = mk(0.0, 1.0, 0.0);
  for (int k = 0; k < 4; ++k) Q.D[k] = mk(0.0, 0.0, 0.0);
  Q.D[0] = mk(0.0, 0.0, -1.0);
  return Q;
}

int main() {
  const Quad Q = unit_quad(0.2), Qout = unit_quad(2.0);
  int fails = 0;
  // 1. (s - 0.5)^5 (s - 2): a fivefold root.  Within about 1e-3 of it the
  //    computed Bernstein coefficients are rounding noise of either sign, so
  //    the subdivision keeps isolating spurious sign changes there; none is a
  //    contact (the vertex is outside the triangle), and the search runs out
  //    of its interval budget before it has covered that region.
  {
    double f[7];
    // (s - 0.5)^5 = sum_k C(5,k) s^k (-0.5)^(5-k), times (s - 2)
    const double b5[6] = {1, 5, 10, 10, 5, 1};
    double g[6];
    for (int k = 0; k <= 5; ++k) g[k] = b5[k] * std::pow(-0.5, 5 - k);
    for (int k = 0; k <= 6; ++k) f[k] = (k >= 1 ? g[k - 1] : 0.0) - 2.0 * (k <= 5 ? g[k] : 0.0);
    int visits = 0, deg = 0, exh = 0;
    double s = -1.0;
    const int hit = search_in<6>(Qout, f, 0.0, 1.0, &s, &visits, &deg, &exh);
    std::printf("fivefold: hit=%d visits=%d deg=%d exh=%d\n", hit, visits, deg, exh);
    if (exh != 1 || hit != 0 || visits <= kMaxSearchVisits) ++fails;
  }
  // 2. A simple root of the same search: found, nothing exhausted, the
  //    vertex plane z = 0.5 - s meets d = 0.1 at s = 0.4 (F = g^2 - d^2 q).
  {
    double f[7];
    const double d = 0.1;
    poly_coeffs<6>(Q, d, f);
    int deg = 0, exh = 0, within = 0;
    double s = -1.0;
    const int hit = earliest<6>(Q, d, &s, &within, &deg, &exh);
    std::printf("simple: hit=%d s=%.17g deg=%d exh=%d\n", hit, s, deg, exh);
    if (hit != 1 || exh != 0 || std::fabs(s - 0.4) > 1e-15) ++fails;
  }
  std::printf(fails ? "FAIL\n" : "OK\n");
  return fails ? 1 : 0;
}
