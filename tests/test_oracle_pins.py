"""Pins of the CPU oracle against facts fixed outside it.

Each test compares the oracle with something that does not share its code:
the defining property of directed rounding, an independent numpy
sort-and-sweep, exact rational evaluation, closed-form times of impact, and
exact-rational root isolation on tiny inputs.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
import scenes
from helpers import q24, numpy_boxes, numpy_sweep_pairs
import exact_ccd

DELTA = 1e-6
U = 2.0 ** -53
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# --------------------------------------------------------------------------- #
# Box rounding (Sec. 5.1): lo = largest float <= x, hi = smallest float >= x.  #
# --------------------------------------------------------------------------- #
def _special_doubles(rng, n):
    parts = [
        rng.normal(size=n),
        rng.normal(size=n) * 1e30,
        rng.normal(size=n) * 1e-40,      # float32 subnormal range
        rng.normal(size=n) * 1e-320,     # double subnormals
        rng.normal(size=n).astype(np.float32).astype(np.float64),  # exactly representable
        np.array([0.0, -0.0, 3.4028234663852886e38, -3.4028234663852886e38, 3.5e38, -3.5e38,
                  1.401298464324817e-45, -1.401298464324817e-45, 7.0e-46, -7.0e-46, 1e300, -1e300]),
    ]
    f = rng.normal(size=n).astype(np.float32)
    mid = (f.astype(np.float64) + np.nextafter(f, np.float32(np.inf)).astype(np.float64)) / 2
    parts.append(mid)  # halfway cases
    return np.concatenate(parts)


def test_box_rounding_is_tight_and_outward():
    rng = np.random.default_rng(7)
    x = _special_doubles(rng, 20000)
    V = np.zeros((len(x), 3))
    V[:, 0] = x
    lo, hi = oracle.boxes(V, V, np.zeros((0, 2), np.int32), np.zeros((0, 3), np.int32))
    lo, hi = lo[:, 0], hi[:, 0]
    big = np.float32(3.4028235e38)
    np.seterr(over="ignore")
    assert np.all(lo.astype(np.float64) <= x) and np.all(hi.astype(np.float64) >= x)
    up = np.nextafter(lo, np.float32(np.inf)).astype(np.float64)
    dn = np.nextafter(hi, np.float32(-np.inf)).astype(np.float64)
    ok_lo = (up > x) | ((lo == big) & (x > float(big)))
    ok_hi = (dn < x) | ((hi == -big) & (x < -float(big)))
    assert np.all(ok_lo), x[~ok_lo][:5]
    assert np.all(ok_hi), x[~ok_hi][:5]


def test_boxes_match_numpy_on_scene():
    s = scenes.two_spheres()
    lo, hi = oracle.boxes(s.V0, s.V1, s.E, s.F)
    nlo, nhi = numpy_boxes(s.V0, s.V1, s.E, s.F)
    assert np.array_equal(lo, nlo) and np.array_equal(hi, nhi)


# --------------------------------------------------------------------------- #
# Broad phase: brute force vs an independent sort-and-sweep.                  #
# --------------------------------------------------------------------------- #
@pytest.mark.parametrize("make", [
    lambda: scenes.two_spheres(),
    lambda: scenes.cloth_on_sphere(n=20, sphere_subdivisions=2),
    lambda: scenes.tiny_random_scene(3, n_tris=40, extent=1.0, motion=0.5),
    lambda: scenes.tiny_random_scene(4, n_tris=25, extent=0.3, motion=0.2, dyadic_bits=3),
])
def test_broad_matches_independent_sweep(make):
    s = make()
    vf, ee = oracle.broad(s.V0, s.V1, s.E, s.F)
    for axis in (0, 2):
        svf, see = numpy_sweep_pairs(s.V0, s.V1, s.E, s.F, axis=axis)
        assert np.array_equal(vf, svf)
        assert np.array_equal(ee, see)


def test_broad_pair_rules():
    s = scenes.cloth_on_sphere(n=16, sphere_subdivisions=1)
    vf, ee = oracle.broad(s.V0, s.V1, s.E, s.F)
    assert len(vf) and len(ee)
    assert not np.any(s.F[vf[:, 1]] == vf[:, [0]])           # no vertex of its own face
    assert np.all(ee[:, 0] < ee[:, 1])
    e0, e1 = s.E[ee[:, 0]], s.E[ee[:, 1]]
    assert not np.any((e0[:, :, None] == e1[:, None, :]).any(axis=(1, 2)))  # no shared endpoint
    assert len(np.unique(vf, axis=0)) == len(vf) and len(np.unique(ee, axis=0)) == len(ee)


# --------------------------------------------------------------------------- #
# C_eps: the float64 evaluation stays within eps of the exact value.          #
# --------------------------------------------------------------------------- #
def _exact_F(kind, q, t, u, v):
    X0 = [[Fraction(float(q[3 * k + a])) for a in range(3)] for k in range(4)]
    X1 = [[Fraction(float(q[12 + 3 * k + a])) for a in range(3)] for k in range(4)]
    t, u, v = Fraction(t), Fraction(u), Fraction(v)
    P = [[X0[k][a] + t * (X1[k][a] - X0[k][a]) for a in range(3)] for k in range(4)]
    if kind == 0:
        return [P[0][a] - P[1][a] - u * (P[2][a] - P[1][a]) - v * (P[3][a] - P[1][a]) for a in range(3)]
    return [P[0][a] + u * (P[1][a] - P[0][a]) - P[2][a] - v * (P[3][a] - P[2][a]) for a in range(3)]


def _random_queries(rng, n):
    out = []
    for i in range(n):
        mode = i % 4
        if mode == 0:
            q = rng.normal(size=24)
        elif mode == 1:  # large offset, tiny motion: cancellation
            q = 2.0 ** rng.integers(-60, 61) * (1.0 + 1e-9 * rng.normal(size=24))
        elif mode == 2:  # mixed magnitudes per point
            q = rng.normal(size=24) * 2.0 ** rng.integers(-60, 61, size=24)
        else:  # everything near the axis maximum
            q = 2.0 ** rng.integers(-20, 21) * (1.0 - 1e-3 * rng.random(size=24)) * rng.choice([-1, 1], size=24)
        out.append(q)
    return out


@pytest.mark.parametrize("kind", [0, 1])
def test_eps_bounds_rounding_error(kind):
    rng = np.random.default_rng(11 + kind)
    worst = 0.0
    bound = 34.0 if kind == 0 else 26.0
    for q in _random_queries(rng, 400):
        eps = oracle.eps(kind, q)
        M = np.abs(q.reshape(8, 3)).max(axis=0)
        for _ in range(4):
            lv = rng.integers(0, 53, size=3)
            n = [rng.integers(0, 2 ** int(l)) if l > 0 else 0 for l in lv]
            c = rng.integers(0, 2, size=3)
            tuv = [Fraction(int(n[k]) + int(c[k]), 2 ** int(lv[k])) for k in range(3)]
            got = oracle.eval_F(kind, q, *[float(x) for x in tuv])
            ex = _exact_F(kind, q, *tuv)
            for a in range(3):
                err = abs(Fraction(float(got[a])) - ex[a])
                assert err <= Fraction(float(eps[a])), (kind, a, float(err), eps[a])
                if M[a] > 0:
                    worst = max(worst, float(err / (Fraction(U) * Fraction(float(M[a])))))
    assert worst <= bound, worst


def _exact_F_scaled(kind, X, nt, lt, nu, lu, nv, lv, a):
    """Exact F on axis a at (nt 2^-lt, nu 2^-lu, nv 2^-lv), times 2^(lt + lu + lv), from the integer
    coordinates X (every input times a common power of two)."""
    P = [X[3 * k + a] * (1 << lt) + nt * (X[12 + 3 * k + a] - X[3 * k + a]) for k in range(4)]
    if kind == 0:  # p - a - u (b - a) - v (c - a)
        return ((P[0] - P[1]) << (lu + lv)) - ((nu * (P[2] - P[1])) << lv) - ((nv * (P[3] - P[1])) << lu)
    # a0 + u (a1 - a0) - b0 - v (b1 - b0)
    return ((P[0] - P[2]) << (lu + lv)) + ((nu * (P[1] - P[0])) << lv) - ((nv * (P[3] - P[2])) << lu)


def _adversarial_queries(rng, n):
    """The four modes of _random_queries plus points clustered within a few ulps of each other far from the
    origin (cancellation in every difference) and coordinates of both signs at the axis maximum."""
    base = _random_queries(rng, n)
    for i in range(0, n, 5):
        c = 2.0 ** rng.integers(-40, 41) * rng.choice([-1, 1], size=3)
        q = np.tile(c, 8) * (1.0 + 2.0 ** -50 * rng.integers(-8, 9, size=24))
        base[i] = q
    for i in range(2, n, 5):
        M = 2.0 ** rng.integers(-30, 31)
        base[i] = M * rng.choice([-1.0, 1.0, -(1 - 2.0 ** -52), 1 - 2.0 ** -52], size=24)
    return base


@pytest.mark.slow
@pytest.mark.parametrize("kind", [0, 1])
def test_eps_bounds_rounding_error_large(kind):
    """10^5 corners per kind (25,000 queries x 4 random dyadic corners, 3 axes each) in exact integer
    arithmetic: |fl(F) - F| <= eps_a everywhere, and the worst error stays below the derived bound (34 uM for
    vertex-face, 26 uM for edge-edge), so eps (36 uM, 28 uM) keeps a margin above every observed error."""
    rng = np.random.default_rng(101 + kind)
    bound = 34.0 if kind == 0 else 26.0
    worst = 0.0
    n_corners = 0
    for q in _adversarial_queries(rng, 25000):
        eps = oracle.eps(kind, q)
        M = np.abs(q.reshape(8, 3)).max(axis=0)
        ratios = [x.as_integer_ratio() for x in q.tolist()]
        S = max(d.bit_length() - 1 for _, d in ratios)
        X = [m << (S - (d.bit_length() - 1)) for m, d in ratios]
        for _ in range(4):
            lv = [int(x) for x in rng.integers(0, 53, size=3)]
            num = [int(rng.integers(0, 2 ** l)) + int(rng.integers(0, 2)) if l > 0 else int(rng.integers(0, 2))
                   for l in lv]
            got = oracle.eval_F(kind, q, *[num[k] / 2 ** lv[k] for k in range(3)])
            scale = S + lv[0] + lv[1] + lv[2]
            for a in range(3):
                ex = Fraction(_exact_F_scaled(kind, X, num[0], lv[0], num[1], lv[1], num[2], lv[2], a), 1 << scale)
                err = abs(Fraction(float(got[a])) - ex)
                assert err <= Fraction(float(eps[a])), (kind, a, float(err), eps[a])
                if M[a] > 0:
                    worst = max(worst, float(err / (Fraction(U) * Fraction(float(M[a])))))
            n_corners += 1
    assert n_corners == 100000
    print(f"kind {kind}: worst |fl(F) - F| / (u M) = {worst:.3f} (bound {bound})")
    assert worst <= bound, worst


# --------------------------------------------------------------------------- #
# Split levels: smallest m with 3 L 2^-m <= delta.                            #
# --------------------------------------------------------------------------- #
def test_levels_needed_closed_form():
    tri = [(0, 0, 0), (1, 0, 0), (0, 1, 0)]
    q = q24([(0.25, 0.25, 1.0)] + tri, [(0.25, 0.25, 0.0)] + tri)  # L_t = L_u = L_v = 1
    for delta in (1e-6, 3 * 2.0 ** -20, 1e-3, 3.0, 10.0):
        want = 0
        while Fraction(3) * Fraction(1, 2 ** want) > Fraction(delta):
            want += 1
        assert list(oracle.levels_needed(0, q, delta)) == [want] * 3
    # L_t = 2 (vertex moves by 2), L_u = 4, L_v = 0.5
    q = q24([(0, 0, 2.0), (0, 0, 0), (4, 0, 0), (0, 0.5, 0)], [(0, 0, 0.0), (0, 0, 0), (4, 0, 0), (0, 0.5, 0)])
    m = oracle.levels_needed(0, q, 1e-6)
    for k, L in enumerate((2, 4, Fraction(1, 2))):
        want = 0
        while 3 * Fraction(L) / 2 ** want > Fraction(1e-6):
            want += 1
        assert m[k] == want


def _true_L(kind, q):
    """Sup over [0,1]^3 of |dF/dt|, |dF/du|, |dF/dv| (max over axes), from the derivatives' closed forms in
    exact rationals.  Each derivative is affine in every parameter it depends on, so its extremes are at the
    corners:
      VF: dF/dt = dp - (1-u-v) da - u db - v dc;  dF/du = -(b(t) - a(t));  dF/dv = -(c(t) - a(t))
      EE: dF/dt = (1-u) da0 + u da1 - (1-v) db0 - v db1;  dF/du = a1(t) - a0(t);  dF/dv = -(b1(t) - b0(t))"""
    X0 = [[Fraction(float(q[3 * k + a])) for a in range(3)] for k in range(4)]
    X1 = [[Fraction(float(q[12 + 3 * k + a])) for a in range(3)] for k in range(4)]
    d = [[X1[k][a] - X0[k][a] for a in range(3)] for k in range(4)]
    Lt = Lu = Lv = Fraction(0)
    for a in range(3):
        for u in (0, 1):
            for v in (0, 1):
                if kind == 0:
                    g = d[0][a] - (1 - u - v) * d[1][a] - u * d[2][a] - v * d[3][a]
                else:
                    g = (1 - u) * d[0][a] + u * d[1][a] - (1 - v) * d[2][a] - v * d[3][a]
                Lt = max(Lt, abs(g))
        for X in (X0, X1):
            if kind == 0:
                Lu, Lv = max(Lu, abs(X[2][a] - X[1][a])), max(Lv, abs(X[3][a] - X[1][a]))
            else:
                Lu, Lv = max(Lu, abs(X[1][a] - X[0][a])), max(Lv, abs(X[3][a] - X[2][a]))
    return Lt, Lu, Lv


def _exact_m(L, delta):
    m = 0
    while 3 * L / 2 ** m > Fraction(delta):
        m += 1
    return m


# Edge-edge queries (a0, a1, b0, b1 at t=0, then at t=1) whose derivative bounds are attained (the edges'
# velocities have opposite signs on the axis of the largest one), each with a different largest L, and with
# edges that stretch or shrink so that the length at t=0 and at t=1 differ by more than a factor of 2.
EE_L_CASES = [
    # a translates by +2 in z, b static: L_t = 2, L_u = |a1 - a0| = 4, L_v = |b1 - b0| = 1/2
    ([(0, 0, 0), (4, 0, 0), (1, -0.25, 1), (1, 0.25, 1)], [(0, 0, 2), (4, 0, 2), (1, -0.25, 1), (1, 0.25, 1)],
     (2, 4, 0.5)),
    # a1 moves (+4, 0, +3), b moves -1 in z with b1 pulled back in y: L_t = 3u + 1 -> 4 (z) and 4u (x),
    # L_u = |a1 - a0| grows from 4 to 8 (x), L_v = |b1 - b0| shrinks from 1 to 1/4 (y)
    ([(0, 0, 0), (4, 0, 0), (1, -0.5, 1), (1, 0.5, 1)], [(0, 0, 0), (8, 0, 3), (1, -0.5, 0), (1, -0.25, 0)],
     (4, 8, 1)),
    # the roles of the two edges swapped: L_u = 1/4 .. 1/2, L_v = 8 .. 16, L_t = 1.25 + 8 (y: a1 moves +1.25,
    # b0 -8)
    ([(0, 0, 0), (0, 0.25, 0), (-4, 1, 0), (4, 1, 0)], [(0, 1, 0), (0, 1.5, 0), (-8, -7, 0), (8, 1, 0)],
     (9.25, 0.5, 16)),
    # a shrinks from length 8 to 2 while a0 rises by 1: L_t = 6 (x, u = 1), L_u = 8 at t=0, L_v = 2
    ([(0, 0, 0), (8, 0, 0), (1, -1, 0.5), (1, 1, 0.5)], [(0, 0, 1), (2, 0, 1), (1, -1, 0.5), (1, 1, 0.5)],
     (6, 8, 2)),
]


@pytest.mark.parametrize("case", range(len(EE_L_CASES)))
def test_levels_needed_closed_form_edge_edge(case):
    p0, p1, want_L = EE_L_CASES[case]
    q = q24(p0, p1)
    L = _true_L(1, q)
    assert L == tuple(Fraction(x) for x in want_L), L
    for delta in (1e-6, 2.0 ** -20, 1e-3, 0.7):
        m = oracle.levels_needed(1, q, delta)
        assert list(m) == [_exact_m(x, delta) for x in L], (delta, list(m), L)


def test_levels_needed_closed_form_vertex_face_moving():
    """p +1, a +1, b -2, c -1 in z: at (u, v) = (1, 1) dF/dt = dp + da - db - dc = 5, the bound's value;
    |b - a| grows from 2 to 3 and |c - a| from 1/2 to 2."""
    q = q24([(0.25, 0.25, 1), (0, 0, 0), (2, 0, 0), (0, 0.5, 0)], [(0.25, 0.25, 2), (0, 0, 1), (2, 0, -2), (0, 1, -1)])
    L = _true_L(0, q)
    assert L == (5, 3, 2), L
    for delta in (1e-6, 1e-3, 0.7):
        m = oracle.levels_needed(0, q, delta)
        assert list(m) == [_exact_m(x, delta) for x in L], (delta, list(m), L)


# --------------------------------------------------------------------------- #
# Closed-form times of impact.                                                #
# --------------------------------------------------------------------------- #
TRI = [(0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0)]


def vf_head_on(h, s, p=(0.25, 0.25), shift=0.0, perm=(0, 1, 2), tri_speed=0.0):
    def P(x):
        x = np.asarray(x, float) + shift
        return x[list(perm)]
    pts0 = [P((p[0], p[1], h))] + [P(c) for c in TRI]
    pts1 = [P((p[0], p[1], h - s))] + [P((c[0], c[1], c[2] + tri_speed)) for c in TRI]
    return q24(pts0, pts1), h / (s + tri_speed)


def ee_crossing(h, s, shift=0.0, perm=(0, 1, 2)):
    def P(x):
        x = np.asarray(x, float) + shift
        return x[list(perm)]
    a0, a1 = (-1.0, 0.0, h), (1.0, 0.0, h)
    b0, b1 = (0.0, -1.0, 0.0), (0.0, 1.0, 0.0)
    pts0 = [P(a0), P(a1), P(b0), P(b1)]
    pts1 = [P((-1.0, 0.0, h - s)), P((1.0, 0.0, h - s)), P(b0), P(b1)]
    return q24(pts0, pts1), h / s


CASES = []
for h, s in [(0.25, 1.0), (0.5, 1.0), (0.3, 0.9), (1e-3, 1.0), (0.0, 1.0), (1.0, 1.0), (0.75, 0.8)]:
    CASES.append(("vf", 0) + vf_head_on(h, s) + (s,))
    CASES.append(("ee", 1) + ee_crossing(h, s) + (s,))
for k in (3, 10, 20, 30):
    CASES.append(("vf+2^%d" % k, 0) + vf_head_on(0.25, 1.0, shift=2.0 ** k) + (1.0,))
    CASES.append(("ee+2^%d" % k, 1) + ee_crossing(0.25, 1.0, shift=2.0 ** k) + (1.0,))
for perm in ((2, 0, 1), (1, 2, 0)):
    CASES.append(("vf perm", 0) + vf_head_on(0.4, 1.0, perm=perm) + (1.0,))
    CASES.append(("ee perm", 1) + ee_crossing(0.4, 1.0, perm=perm) + (1.0,))
CASES.append(("vf on edge", 0) + vf_head_on(0.5, 1.0, p=(0.5, 0.0)) + (1.0,))
# the vertex lands on the hypotenuse u + v = 1 (the face's edge b-c), at its middle and near either end
for pu in (0.5, 0.25, 0.875):
    CASES.append(("vf on hypotenuse u=%g" % pu, 0) + vf_head_on(0.4, 1.0, p=(pu, 1.0 - pu)) + (1.0,))
CASES.append(("vf on corner b", 0) + vf_head_on(0.5, 1.0, p=(1.0, 0.0)) + (1.0,))
CASES.append(("vf on corner c", 0) + vf_head_on(0.5, 1.0, p=(0.0, 1.0)) + (1.0,))
CASES.append(("vf on corner", 0) + vf_head_on(0.5, 1.0, p=(0.0, 0.0)) + (1.0,))
CASES.append(("vf both move", 0) + vf_head_on(0.5, 0.5, tri_speed=0.5) + (1.0,))


@pytest.mark.parametrize("name,kind,q,te,speed", CASES, ids=[c[0] for c in CASES])
def test_closed_form_toi(name, kind, q, te, speed):
    hit, toi, n_enq, n_eval = oracle.query(kind, q, DELTA, 10 ** 6)
    eps = oracle.eps(kind, q).max()
    assert hit
    assert toi <= te
    assert te - toi <= (DELTA + 2 * eps) / speed + 1e-15, (te, toi)
    assert n_enq <= 10 ** 6


@pytest.mark.parametrize("case", ["vf beside", "ee parallel apart", "ee skew apart", "vf static far",
                                  "vf past hypotenuse", "vf past hypotenuse near b", "vf past corner c"])
def test_clear_misses(case):
    if case == "vf beside":
        kind, q = 0, q24([(2, 2, 1)] + TRI, [(2, 2, -1)] + TRI)
    elif case.startswith("vf past"):
        # the vertex crosses the face's plane just outside the triangle, 2^-7 beyond u + v = 1 (a clearance
        # of ~0.0055, far above delta and C_eps), so the plane is hit but the triangle is not
        pu, pv = {"vf past hypotenuse": (0.5, 0.5), "vf past hypotenuse near b": (0.875, 0.125),
                  "vf past corner c": (0.0, 1.0)}[case]
        pu, pv = pu + 2.0 ** -8, pv + 2.0 ** -8
        kind, q = 0, q24([(pu, pv, 0.4)] + TRI, [(pu, pv, -0.6)] + TRI)
    elif case == "ee parallel apart":
        kind, q = 1, q24([(0, 0, 1), (1, 0, 1), (0, 0.5, 0), (1, 0.5, 0)],
                         [(0, 0, 0.0), (1, 0, 0.0), (0, 0.5, 0), (1, 0.5, 0)])
    elif case == "ee skew apart":
        kind, q = 1, q24([(-1, 0, 1), (1, 0, 1), (3, -1, 0), (3, 1, 0)],
                         [(-1, 0, -1), (1, 0, -1), (3, -1, 0), (3, 1, 0)])
    else:
        kind, q = 0, q24([(0.2, 0.2, 0.5)] + TRI, [(0.2, 0.2, 0.5)] + TRI)
    hit, toi, _, _ = oracle.query(kind, q, DELTA, 10 ** 6)
    assert not hit and toi == np.inf


def _parallel_edges(h=0.5, s=1.0):
    a = [(0.0, 0.0, h), (1.0, 0.0, h)]
    b = [(0.25, 0.0, 0.0), (1.25, 0.0, 0.0)]
    q = q24(a + b, [(0.0, 0.0, h - s), (1.0, 0.0, h - s)] + b)
    return q, h / s


@pytest.mark.parametrize("max_iter", [1, 10, 1000, 10 ** 6])
def test_cap_on_degenerate_parallel_edges(max_iter):
    q, te = _parallel_edges()
    hit, toi, n_enq, n_eval = oracle.query(1, q, DELTA, max_iter)
    assert hit and toi <= te
    if max_iter < 10 ** 6:
        assert n_enq > max_iter  # the cap was reached
    assert n_eval <= 2 * max_iter + 2


def test_delta_huge_accepts_root_interval():
    q, te = vf_head_on(0.25, 1.0)
    hit, toi, n_enq, n_eval = oracle.query(0, q, 100.0, 10 ** 6)
    assert hit and toi == 0.0 and n_eval == 1 and n_enq == 0


# --------------------------------------------------------------------------- #
# Exact rational pins: the printed cubic, and brute force on tiny inputs.     #
# --------------------------------------------------------------------------- #
def test_root_isolator_on_printed_cubic():
    lines = [ln for ln in open(os.path.join(GOLDEN, "root_example_cubic.txt")) if not ln.startswith("#")]
    coeffs = [int(x) for x in lines if x.strip()]
    lo, hi = exact_ccd.nth_real_root_interval(coeffs, 2)
    approx = sorted(r.real for r in np.roots([float(c) for c in coeffs]) if abs(r.imag) < 1e-9)[1]
    assert float(lo) <= approx + 1e-9 and approx - 1e-9 <= float(hi)
    assert hi - lo < 1e-20 and 0 < lo and hi < 1  # a valid time of impact
    f = exact_ccd.sp.Poly(coeffs, exact_ccd.T, domain="QQ")
    fs, roots = exact_ccd._roots_in_unit(f)
    assert len(roots) == 2  # 0.1233... and 0.8579... lie in [0, 1]


def _exact_cases(seed, n_tris, bits):
    s = scenes.tiny_random_scene(seed, n_tris=n_tris, extent=0.5, motion=1.0, dyadic_bits=bits)
    vf, ee = oracle.all_pairs(s.E, s.F, s.nv)
    return s, vf, ee


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_tiny_scenes_against_exact_toi(seed):
    s, vf, ee = _exact_cases(seed, 5, 4)
    hit, toi, _, _, tmin = oracle.narrow(s.V0, s.V1, s.E, s.F, vf, ee, DELTA, 10 ** 6)
    n_true = n_undecided = n_fp = 0
    errs = []
    for i in range(len(vf) + len(ee)):
        if i < len(vf):
            v, f = vf[i]
            ids = [v, *s.F[f]]
            kind = 0
        else:
            e, g = ee[i - len(vf)]
            ids = [*s.E[e], *s.E[g]]
            kind = 1
        q = np.concatenate([s.V0[ids].reshape(-1), s.V1[ids].reshape(-1)])
        ex = exact_ccd.exact_toi(kind, q)
        if ex == exact_ccd.UNDECIDED:
            n_undecided += 1
            continue
        if ex is None:
            n_fp += int(hit[i])
            continue
        n_true += 1
        lo, hi = ex
        assert hit[i] == 1, (i, kind)                 # no false negative
        assert toi[i] <= float(hi), (i, toi[i], float(hi))   # never after the exact contact
        errs.append(float(lo) - toi[i])
    assert n_undecided == 0
    assert n_true >= 5
    assert n_fp <= n_true // 4      # false positives only for near misses
    assert np.median(errs) < 1e-4


# --------------------------------------------------------------------------- #
# The split rule goes on past m_k while the inclusion box is not narrower     #
# than delta (Alg. 3 splits until w(B) < delta; m_k only ranks dimensions).   #
# --------------------------------------------------------------------------- #
DEEP_SEEDS = {0: {1.07e-6: [367, 1129, 1751, 1924, 2207, 2578, 3604], 1e-6: [2886]},
              1: {1.07e-6: [685, 1181, 1570, 1658], 1e-6: [136, 751, 2076, 3970]}}


@pytest.mark.parametrize("kind", [0, 1])
def test_split_levels_pass_m_when_box_stays_wide(kind):
    from helpers import deep_split_query
    for delta, seeds in DEEP_SEEDS[kind].items():
        for seed in seeds:
            q, d = deep_split_query(seed, kind)
            assert d == delta
            m = oracle.levels_needed(kind, q, d)
            hit, toi, n_enq, lv = oracle.query_levels(kind, q, d, 10 ** 6)
            assert max(m) <= 21 and max(lv) > 21, (seed, m, lv)
            assert hit and n_enq < 60000
