"""Exact-arithmetic referee for tiny narrow-phase inputs (pins the oracle).

Independent of the oracle's code: the polynomial is obtained by expanding
the *definition* of the distance condition symbolically in rational
arithmetic (no hand-written coefficient formulas), its real roots in [0,1]
are isolated exactly (sympy's exact real-root isolation), and the inside test
is evaluated exactly at both ends of each isolating interval.

Definitions (Eq. 3.1 with linear trajectories P(s) = X0 + s (X1 - X0)):
  vertex-triangle: g = (P_p - P_a) . ((P_b - P_a) x (P_c - P_a)), q = |n|^2
  edge-edge:       g = (P_c - P_a) . ((P_b - P_a) x (P_e - P_c)), q = |m|^2
  F = g^2 - d^2 q   (d > 0),   F = g (d = 0).
A contact is the earliest s in [0,1] with F(s) = 0 where the closest point
lies inside the triangle (resp. both segments); if F(0) < 0 and the point is
inside at s = 0 the contact is at s = 0.
"""
from fractions import Fraction

import sympy as sp

_s = sp.symbols("s")


def _q(x):
    return sp.Rational(Fraction(float(x)))


def _traj(x0, x1):
    P0 = [sp.Matrix([_q(v) for v in row]) for row in x0]
    P1 = [sp.Matrix([_q(v) for v in row]) for row in x1]
    return P0, P1


def _geom(P, ee):
    if not ee:
        p, a, b, c = P
        e1, e2, w = b - a, c - a, p - a
        n = e1.cross(e2)
        return e1, e2, w, n
    a, b, c, e = P
    ea, eb, w = b - a, e - c, c - a
    m = ea.cross(eb)
    return ea, eb, w, m


def polynomial(x0, x1, ee, d):
    """Exact sympy Poly F(s) and the pieces (g, q) as Polys."""
    P0, P1 = _traj(x0, x1)
    P = [P0[k] + _s * (P1[k] - P0[k]) for k in range(4)]
    u, v, w, n = _geom(P, ee)
    g = sp.expand(w.dot(n))
    q = sp.expand(n.dot(n))
    dd = _q(d)
    F = g if dd == 0 else sp.expand(g ** 2 - dd ** 2 * q)
    return sp.Poly(F, _s), sp.Poly(g, _s), sp.Poly(q, _s)


def _inside_exact(x0, x1, ee, sval):
    P0, P1 = _traj(x0, x1)
    P = [P0[k] + sval * (P1[k] - P0[k]) for k in range(4)]
    u, v, w, n = _geom(P, ee)
    q = n.dot(n)
    if q == 0:
        return None
    if not ee:
        B = w.cross(v).dot(n)
        C = u.cross(w).dot(n)
        return bool(B >= 0 and C >= 0 and B + C <= q)
    U = w.cross(v).dot(n)
    W = w.cross(u).dot(n)
    return bool(0 <= U <= q and 0 <= W <= q)


def earliest(x0, x1, ee=False, d=0.0, eps_bits=60):
    """(hit, s, ambiguous).  `ambiguous` is True when the inside test differs
    at the two ends of an isolating interval (input too close to the edge of
    the triangle/segment for a unique decision at this resolution)."""
    F, g, q = polynomial(x0, x1, ee, d)
    if F.is_zero:
        return False, None, False
    if _q(d) != 0 and F.eval(0) < 0:
        ins = _inside_exact(x0, x1, ee, sp.Integer(0))
        if ins:
            return True, 0.0, False
    if F.degree() <= 0:
        return False, None, False
    ivs = F.intervals(eps=sp.Rational(1, 2 ** eps_bits), inf=0, sup=1)
    ivs = sorted(ivs, key=lambda t: t[0][0])
    for (lo, hi), _mult in ivs:
        a = _inside_exact(x0, x1, ee, sp.Rational(lo))
        b = _inside_exact(x0, x1, ee, sp.Rational(hi))
        if a is None or b is None:
            continue
        if a != b:
            return None, float((lo + hi) / 2), True
        if a:
            return True, float((lo + hi) / 2), False
    return False, None, False
