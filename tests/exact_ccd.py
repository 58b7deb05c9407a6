"""Exact rational time of impact for tiny inputs (a pin of the oracle).

Linear trajectories with rational coordinates.  A vertex-face or edge-edge
contact needs the four points to be coplanar, so the earliest contact time is
the first root in [0, 1] of the coplanarity cubic at which the point lies in
the triangle (or the two segments cross).  Roots are isolated exactly with
sympy (Sturm sequences over the rationals); the sign of each inside-ness
polynomial at an algebraic root is decided exactly by refining the isolating
interval, with common roots detected through polynomial gcds.

Degenerate situations (identically coplanar motion, a triangle or edge pair
that degenerates exactly at the root) are reported as undecided instead of
being guessed.
"""
from fractions import Fraction

import sympy as sp

T = sp.Symbol("t")
UNDECIDED = "undecided"


def _vec(q24, k):
    """Point k of a 24-value query as a linear function of t: (x0, x1) rationals."""
    x0 = [Fraction(float(q24[3 * k + a])) for a in range(3)]
    x1 = [Fraction(float(q24[12 + 3 * k + a])) for a in range(3)]
    return [sp.Rational(x0[a].numerator, x0[a].denominator)
            + T * (sp.Rational(x1[a].numerator, x1[a].denominator) - sp.Rational(x0[a].numerator, x0[a].denominator))
            for a in range(3)]


def _sub(p, q):
    return [p[a] - q[a] for a in range(3)]


def _cross(p, q):
    return [p[1] * q[2] - p[2] * q[1], p[2] * q[0] - p[0] * q[2], p[0] * q[1] - p[1] * q[0]]


def _dot(p, q):
    return p[0] * q[0] + p[1] * q[1] + p[2] * q[2]


def _poly(e):
    return sp.Poly(sp.expand(e), T, domain="QQ")


def _sign_at_root(g, f, lo, hi):
    """Sign of polynomial g at the unique root of square-free f in [lo, hi]."""
    if g.is_zero:
        return 0
    h = sp.gcd(f, g)
    if h.degree() > 0 and h.count_roots(lo, hi) > 0:
        return 0
    lo, hi = sp.Rational(lo), sp.Rational(hi)
    for _ in range(400):
        if g.count_roots(lo, hi) == 0:
            mid = (lo + hi) / 2
            val = g.eval(mid)
            return 1 if val > 0 else -1
        mid = (lo + hi) / 2
        fm = f.eval(mid)
        if fm == 0:
            val = g.eval(mid)
            return 0 if val == 0 else (1 if val > 0 else -1)
        if f.count_roots(lo, mid) > 0:
            hi = mid
        else:
            lo = mid
    raise RuntimeError("sign refinement did not converge")


def _roots_in_unit(f):
    """Isolating intervals (lo, hi) of the distinct real roots of f in [0, 1], ascending."""
    fs = sp.Poly(sp.quo(f, sp.gcd(f, f.diff(T))), T, domain="QQ") if f.degree() > 0 else f
    out = []
    for (lo, hi), _mult in fs.intervals():
        lo, hi = sp.Rational(lo), sp.Rational(hi)
        if hi < 0 or lo > 1:
            continue
        # tighten so the interval is inside [0, 1] or touches it only at a root
        if lo < 0 or hi > 1:
            if lo < 0 and fs.eval(0) == 0:
                out.append((sp.Rational(0), sp.Rational(0)))
                continue
            if hi > 1 and fs.eval(1) == 0:
                out.append((sp.Rational(1), sp.Rational(1)))
                continue
            a, b = max(lo, sp.Rational(0)), min(hi, sp.Rational(1))
            if fs.count_roots(a, b) == 0:
                continue
            lo, hi = a, b
        out.append((lo, hi))
    return fs, out


def exact_toi(kind, q24):
    """Exact earliest contact time in [0, 1] as (lo, hi) rationals bracketing it,
    None for no contact, or UNDECIDED for a degenerate configuration."""
    P = [_vec(q24, k) for k in range(4)]
    if kind == 0:
        p, a, b, c = P
        ba, ca, pa = _sub(b, a), _sub(c, a), _sub(p, a)
        f = _poly(_dot(_cross(ba, ca), pa))
        n = _cross(ba, ca)
        gs = [_poly(_dot(_cross(_sub(b, a), _sub(p, a)), n)),
              _poly(_dot(_cross(_sub(c, b), _sub(p, b)), n)),
              _poly(_dot(_cross(_sub(a, c), _sub(p, c)), n))]
        nn = _poly(_dot(n, n))
    else:
        a0, a1, b0, b1 = P
        ea, eb, w = _sub(a1, a0), _sub(b1, b0), _sub(b0, a0)
        f = _poly(_dot(_cross(ea, eb), w))
        n = _cross(ea, eb)
        nn = _poly(_dot(n, n))
        gu = _poly(_dot(_cross(w, eb), n))
        gv = _poly(_dot(_cross(w, ea), n))
        gs = [gu, nn - gu, gv, nn - gv]
    if f.is_zero:
        return UNDECIDED
    fs, roots = _roots_in_unit(f)
    for lo, hi in roots:
        if lo == hi:
            r = lo
            if nn.eval(r) == 0:
                return UNDECIDED
            if all(g.eval(r) >= 0 for g in gs):
                return (r, r)
            continue
        if _sign_at_root(nn, fs, lo, hi) == 0:
            return UNDECIDED
        if all(_sign_at_root(g, fs, lo, hi) >= 0 for g in gs):
            return (lo, hi)
    return None


def nth_real_root_interval(coeffs, n, width=sp.Rational(1, 10**30)):
    """Isolating interval of the n-th (1-based, ascending) real root of an integer polynomial."""
    f = sp.Poly(coeffs, T, domain="QQ")
    ivs = f.intervals(eps=width)
    (lo, hi), _ = ivs[n - 1]
    return sp.Rational(lo), sp.Rational(hi)
