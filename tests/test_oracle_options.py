"""Pins of the oracle's global-t* mode (Alg. 3 as printed), minimum separation (Sec. 7) and no-zero-TOI
strategy (App. B), and of its initial-distance helper, against closed forms, brute force and the per-pair
oracle whose own pins are in test_oracle_pins.py."""
import numpy as np
import pytest

import oracle
import scenes
from helpers import q24

DELTA = 1e-6
TRI = [(0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0)]


def one_pair_scene(kind, q):
    """A scene holding one query: a lone vertex and a triangle (VF) or two lone edges (EE)."""
    q = np.asarray(q, np.float64).reshape(2, 4, 3)
    V0, V1 = q[0].copy(), q[1].copy()
    if kind == 0:
        return V0, V1, np.zeros((0, 2), np.int32), np.array([[1, 2, 3]], np.int32), \
            np.array([[0, 0]], np.int32), np.zeros((0, 2), np.int32)
    return V0, V1, np.array([[0, 1], [2, 3]], np.int32), np.zeros((0, 3), np.int32), \
        np.zeros((0, 2), np.int32), np.array([[0, 1]], np.int32)


def solve(kind, q, ms=None, no_zero=False, max_iter=10 ** 6, delta=DELTA):
    V0, V1, E, F, vf, ee = one_pair_scene(kind, q)
    h, t, n, _, _ = oracle.narrow(V0, V1, E, F, vf, ee, delta, max_iter,
                                  ms=None if ms is None else [ms], no_zero=no_zero)
    return bool(h[0]), float(t[0]), int(n[0])


# --------------------------------------------------------------------------- global t* (Alg. 3)
@pytest.mark.parametrize("make", [
    lambda: scenes.two_spheres(),
    lambda: scenes.cloth_on_sphere(n=24, sphere_subdivisions=2, seed=5),
    lambda: scenes.tiny_random_scene(5, n_tris=10, extent=0.5, motion=1.0),
    lambda: scenes.tiny_random_scene(6, n_tris=10, extent=0.5, motion=1.0, dyadic_bits=4),
])
def test_global_tstar_equals_per_pair_minimum(make):
    """One t* shared by all pairs prunes intervals starting at or after it.  It never prunes the interval that
    gives the per-pair minimum, so when that minimum comes from a pair that did not hit the cap, Alg. 3's t*
    equals it in every order the pairs are taken in."""
    s = make()
    vf, ee = oracle.broad(s.V0, s.V1, s.E, s.F)
    if len(vf) + len(ee) == 0:
        vf, ee = oracle.all_pairs(s.E, s.F, s.nv)
    h, t, n_enq, _, tmin = oracle.narrow(s.V0, s.V1, s.E, s.F, vf, ee)
    assert not np.any((t == tmin) & (n_enq > 10 ** 6))  # the minimum is not a capped pair's
    rng = np.random.default_rng(len(vf))
    for order in (None, rng.permutation(len(vf) + len(ee)), np.arange(len(vf) + len(ee))[::-1]):
        g, searched = oracle.narrow_global(s.V0, s.V1, s.E, s.F, vf, ee, order=order)
        assert np.float64(g).view(np.int64) == np.float64(tmin).view(np.int64), (g, tmin)


def test_global_tstar_with_capped_pairs_is_conservative():
    """With degenerate (capped) pairs the shared t* is never below the per-pair minimum and never after a true
    contact: parallel edges sliding onto each other (contact from t = 1/2 on)."""
    a = [(0.0, 0.0, 0.5), (1.0, 0.0, 0.5)]
    b = [(0.25, 0.0, 0.0), (1.25, 0.0, 0.0)]
    q = q24(a + b, [(0.0, 0.0, -0.5), (1.0, 0.0, -0.5)] + b)
    V0, V1, E, F, vf, ee = one_pair_scene(1, q)
    for max_iter in (10, 1000):
        _, _, n, _, tmin = oracle.narrow(V0, V1, E, F, vf, ee, DELTA, max_iter)
        assert n[0] > max_iter
        g, _ = oracle.narrow_global(V0, V1, E, F, vf, ee, DELTA, max_iter)
        assert tmin <= g <= 0.5


def test_global_stops_once_tstar_is_zero():
    """A pair in contact at t = 0 makes t* = 0: no later pair is searched."""
    touch = q24([(0.25, 0.25, 0.0)] + TRI, [(0.25, 0.25, 1.0)] + TRI)     # vertex on the face at t = 0
    far = q24([(5.0, 5.0, 1.0)] + TRI, [(5.0, 5.0, -1.0)] + TRI)
    P0 = np.concatenate([touch.reshape(2, 4, 3)[0], far.reshape(2, 4, 3)[0]])
    P1 = np.concatenate([touch.reshape(2, 4, 3)[1], far.reshape(2, 4, 3)[1]])
    F = np.array([[1, 2, 3], [5, 6, 7]], np.int32)
    vf = np.array([[0, 0], [4, 1]], np.int32)
    E = np.zeros((0, 2), np.int32)
    g, searched = oracle.narrow_global(P0, P1, E, F, vf, np.zeros((0, 2), np.int32))
    assert g == 0.0 and searched == 1


# --------------------------------------------------------------------------- minimum separation (Sec. 7)
@pytest.mark.parametrize("h,s,ms", [(0.5, 1.0, 0.1), (0.3, 0.6, 0.05), (1.0, 1.0, 0.25), (0.25, 1.0, 2.0 ** -10)])
def test_min_separation_vertex_face_head_on(h, s, ms):
    """A vertex falling onto the face's interior at speed s from height h first comes within ms of it at
    t = (h - ms) / s.  The enlarged box's boundary is then a whole sheet of (u, v) at that time, so at
    delta = 1e-6 the search hits the cap (reporting the earliest interval left, never after te); at
    delta = 1e-3 it resolves the time to within delta / s."""
    q = q24([(0.25, 0.25, h)] + TRI, [(0.25, 0.25, h - s)] + TRI)
    te = (h - ms) / s
    hit, toi, n_enq = solve(0, q, ms=ms)
    assert hit and toi <= te
    hit, toi, n_enq = solve(0, q, ms=ms, delta=1e-3)
    assert hit and toi <= te and n_enq <= 10 ** 6
    assert te - toi <= 1e-3 / s, (te, toi)


@pytest.mark.parametrize("h,ms", [(0.5, 0.1), (0.75, 0.125)])
def test_min_separation_edge_edge_crossing(h, ms):
    a0, a1, b0, b1 = (-1.0, 0.0, h), (1.0, 0.0, h), (0.0, -1.0, 0.0), (0.0, 1.0, 0.0)
    q = q24([a0, a1, b0, b1], [(-1.0, 0.0, h - 1.0), (1.0, 0.0, h - 1.0), b0, b1])
    te = h - ms
    hit, toi, _ = solve(1, q, ms=ms)
    assert hit and toi <= te
    hit, toi, n_enq = solve(1, q, ms=ms, delta=1e-3)
    assert hit and toi <= te and n_enq <= 10 ** 6 and te - toi <= 1e-3


def test_min_separation_changes_nothing_when_zero_and_keeps_far_pairs_apart():
    q = q24([(0.25, 0.25, 0.5)] + TRI, [(0.25, 0.25, -0.5)] + TRI)
    assert solve(0, q, ms=0.0) == solve(0, q)
    # a vertex passing 0.5 above the face: no hit with ms = 0.4, a hit at t = 0 with ms = 0.6
    q = q24([(0.25, -1.0, 0.5)] + TRI, [(0.25, 2.0, 0.5)] + TRI)
    assert not solve(0, q, ms=0.4)[0]
    hit, toi, _ = solve(0, q, ms=0.6)
    assert hit and toi <= 1.0 / 3.0   # the vertex is over the face from t = 1/3 on


# --------------------------------------------------------------------------- no-zero TOI (App. B)
def test_no_zero_splits_at_zero():
    """A vertex 1e-9 above the face at t = 0, moving down at speed 1 (true contact at t = 1e-9): the plain
    search accepts the first interval at t = 0 (its box is narrower than delta); with the no-zero strategy
    intervals at t = 0 are split on until they are discarded, and the reported time is positive and never
    after the contact."""
    g = 1e-9
    q = q24([(0.25, 0.25, g)] + TRI, [(0.25, 0.25, g - 1.0)] + TRI)
    hit, toi, _ = solve(0, q)
    assert hit and toi == 0.0
    hit, toi, _ = solve(0, q, no_zero=True)
    assert hit and 0.0 < toi <= g


def test_no_zero_true_contact_at_zero_still_reported():
    """Touching at t = 0 exactly: splitting never discards the root, so only the finest level stops it."""
    q = q24([(0.25, 0.25, 0.0)] + TRI, [(0.25, 0.25, 1.0)] + TRI)
    hit, toi, n = solve(0, q, no_zero=True)
    assert hit and toi == 0.0


def test_no_zero_ignores_the_cap_at_zero():
    """The cap does not stop a search while an interval starting at t = 0 is left: with max_iter = 1 the plain
    search stops at once, the no-zero search runs until the intervals at t = 0 are gone."""
    g = 1e-9
    q = q24([(0.25, 0.25, g)] + TRI, [(0.25, 0.25, g - 1.0)] + TRI)
    hit0, toi0, n0 = solve(0, q, max_iter=1)
    hit1, toi1, n1 = solve(0, q, max_iter=1, no_zero=True)
    assert hit0 and hit1 and toi1 > 0.0 and n1 > n0


# --------------------------------------------------------------------------- initial distance
def _d0(kind, q):
    V0, V1, E, F, vf, ee = one_pair_scene(kind, q)
    return float(oracle.initial_distance(V0, E, F, vf, ee)[0])


def vfq(p, tri=TRI):
    return q24([p] + list(tri), [p] + list(tri))


def eeq(a0, a1, b0, b1):
    return q24([a0, a1, b0, b1], [a0, a1, b0, b1])


@pytest.mark.parametrize("q,kind,want", [
    (vfq((0.25, 0.25, 0.75)), 0, 0.75),                       # over the interior: the height
    (vfq((0.25, 0.25, -2.0)), 0, 2.0),
    (vfq((0.5, -0.3, 0.4)), 0, 0.5),                          # beyond edge a-b: 3-4-5 to the edge
    (vfq((1.3, -0.4, 0.0)), 0, 0.5),                          # beyond vertex b, in the plane
    (vfq((0.75, 0.75, 0.0)), 0, np.sqrt(2) / 4),              # beyond the hypotenuse
    (vfq((0.1, 0.2, 0.0)), 0, 0.0),                           # in the face
    (vfq((2.0, 0.0, 0.0), [(0, 0, 0), (1, 0, 0), (0.5, 0, 0)]), 0, 1.0),   # zero-area face: nearest edge
    (eeq((-1, 0, 0.3), (1, 0, 0.3), (0, -1, 0), (0, 1, 0)), 1, 0.3),      # crossing at height 0.3
    (eeq((0, 0, 0), (1, 0, 0), (0, 0.4, 0), (1, 0.4, 0)), 1, 0.4),        # parallel
    (eeq((0, 0, 0), (1, 0, 0), (1.5, 0, 0), (3, 0, 0)), 1, 0.5),          # collinear, apart
    (eeq((0, 0, 0), (1, 0, 0), (2, -1, 0.0), (2, 1, 0.0)), 1, 1.0),       # nearest at an endpoint
    (eeq((0, 0, 0), (0, 0, 0), (3, 4, 0), (3, 4, 0)), 1, 5.0),            # zero-length edges
    (eeq((-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0)), 1, 0.0),          # intersecting
])
def test_initial_distance_closed_form(q, kind, want):
    assert abs(_d0(kind, q) - want) <= 1e-15 * max(1.0, want)


@pytest.mark.parametrize("kind", [0, 1])
def test_initial_distance_brute_force(kind):
    """Random primitives: d0 is at most every sampled distance and within the sampling resolution of the
    smallest one (1/64 steps of the parameters)."""
    rng = np.random.default_rng(40 + kind)
    s = np.linspace(0.0, 1.0, 65)
    for _ in range(40):
        P = rng.normal(size=(4, 3))
        q = q24(P, P)
        d = _d0(kind, q)
        if kind == 0:
            u, v = np.meshgrid(s, s)
            keep = (u + v) <= 1.0
            u, v = u[keep], v[keep]
            pts = P[1] + u[:, None] * (P[2] - P[1]) + v[:, None] * (P[3] - P[1])
            dist = np.linalg.norm(pts - P[0], axis=1)
            span = np.linalg.norm(P[2] - P[1]) + np.linalg.norm(P[3] - P[1])
        else:
            u, v = np.meshgrid(s, s)
            A = P[0] + u.reshape(-1, 1) * (P[1] - P[0])
            B = P[2] + v.reshape(-1, 1) * (P[3] - P[2])
            dist = np.linalg.norm(A - B, axis=1)
            span = np.linalg.norm(P[1] - P[0]) + np.linalg.norm(P[3] - P[2])
        assert d <= dist.min() + 1e-12
        assert dist.min() - d <= span / 64


# --------------------------------------------------------------------------- timing sample of the broad phase
def test_broad_sample_covers_its_share_of_rows():
    """stride 1 is the whole brute force (same pair counts, every box test); larger strides run a part of the rows
    and never find more pairs."""
    s = scenes.cloth_on_sphere(n=20, sphere_subdivisions=2, seed=3)
    vf, ee = oracle.broad(s.V0, s.V1, s.E, s.F)
    nvf, nee, tvf, tee = oracle.broad_sample(s.V0, s.V1, s.E, s.F, 1)
    assert (nvf, nee) == (len(vf), len(ee))
    assert tvf == s.nv * s.nf and tee == s.ne * (s.ne - 1) / 2
    nvf4, nee4, tvf4, tee4 = oracle.broad_sample(s.V0, s.V1, s.E, s.F, 4)
    assert nvf4 <= len(vf) and nee4 <= len(ee)
    assert 0.15 < tvf4 / tvf < 0.35 and 0.15 < tee4 / tee < 0.35
