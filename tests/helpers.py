"""Shared test helpers: query construction and an independent numpy sweep."""
import numpy as np


def q24(points0, points1):
    """24-value query from 4 points at t=0 and the same 4 points at t=1."""
    a = np.asarray(points0, dtype=np.float64).reshape(4, 3)
    b = np.asarray(points1, dtype=np.float64).reshape(4, 3)
    return np.concatenate([a.reshape(-1), b.reshape(-1)])


def numpy_boxes(V0, V1, E, F):
    """Outward-rounded float32 boxes computed with numpy only (vertices, edges, faces)."""
    def outward(mn, mx):
        lo = mn.astype(np.float32)
        lo = np.where(lo.astype(np.float64) > mn, np.nextafter(lo, np.float32(-np.inf)), lo)
        hi = mx.astype(np.float32)
        hi = np.where(hi.astype(np.float64) < mx, np.nextafter(hi, np.float32(np.inf)), hi)
        return lo.astype(np.float32), hi.astype(np.float32)

    parts = []
    for ids in (np.arange(len(V0))[:, None], np.asarray(E), np.asarray(F)):
        X = np.concatenate([V0[ids], V1[ids]], axis=1)  # (n, 2k, 3)
        parts.append(outward(X.min(axis=1), X.max(axis=1)))
    lo = np.concatenate([p[0] for p in parts])
    hi = np.concatenate([p[1] for p in parts])
    return lo, hi


def numpy_sweep_pairs(V0, V1, E, F, axis=0):
    """Candidate pairs by sort-and-sweep along one axis (independent of the oracle's brute force)."""
    lo, hi = numpy_boxes(V0, V1, E, F)
    nv, ne = len(V0), len(E)
    E = np.asarray(E)
    F = np.asarray(F)
    order = np.argsort(lo[:, axis], kind="stable")
    slo = lo[order, axis]
    ends = np.searchsorted(slo, hi[order, axis], side="right")
    vf, ee = set(), set()
    for r in range(len(order)):
        i = order[r]
        js = order[r + 1:ends[r]]
        if len(js) == 0:
            continue
        ok = np.all((lo[i] <= hi[js]) & (lo[js] <= hi[i]), axis=1)
        for j in js[ok]:
            a, b = (i, j) if i < j else (j, i)
            if a < nv and b >= nv + ne:
                f = b - nv - ne
                if a not in F[f]:
                    vf.add((a, f))
            elif nv <= a < nv + ne and nv <= b < nv + ne:
                e, g = a - nv, b - nv
                if len({*E[e], *E[g]}) == 4:
                    ee.add((e, g))
    vf = np.array(sorted(vf), dtype=np.int32).reshape(-1, 2)
    ee = np.array(sorted(ee), dtype=np.int32).reshape(-1, 2)
    return vf, ee


def deep_split_query(seed, kind):
    """A query with edges and motion of ~0.69 far from the origin (2^28..2^33).

    At delta ~1e-6 its split levels m_k come out at most 21, but float64
    rounding of coordinates that large keeps the inclusion box at least an ulp
    of 2^33 (~2e-6) wide, so the search goes on splitting past m_k.  Returns
    (q24, delta).  Edge-edge queries move each edge rigidly.
    """
    rng = np.random.default_rng(seed)
    off = 2.0 ** int(rng.integers(28, 34))
    delta = float(rng.choice([1e-6, 1.07e-6, 2e-6]))
    s = 0.69
    pts0 = rng.uniform(-s / 2, s / 2, size=(4, 3))
    mot = rng.uniform(-s / 2, s / 2, size=(4, 3)) * rng.uniform(0, 1)
    if kind == 1:
        mot[0] = mot[1]
        mot[2] = mot[3]
    return q24(pts0 + off, pts0 + mot + off), delta


def scene_of_queries(vf_queries, ee_queries):
    """A scene of disconnected primitives holding the given queries, and its pairs.

    Each vertex-face query (24 values: p, a, b, c at t=0 then t=1) becomes a
    lone vertex and a triangle, each edge-edge query (a0, a1, b0, b1) two lone
    edges.  Returns (V0, V1, E, F, vf, ee) with the pairs in query order."""
    P0, P1, E, F, vf, ee = [], [], [], [], [], []
    for q in vf_queries:
        q = np.asarray(q, np.float64).reshape(2, 4, 3)
        b = len(P0)
        P0 += list(q[0])
        P1 += list(q[1])
        F.append((b + 1, b + 2, b + 3))
        vf.append((b, len(F) - 1))
    for q in ee_queries:
        q = np.asarray(q, np.float64).reshape(2, 4, 3)
        b = len(P0)
        P0 += list(q[0])
        P1 += list(q[1])
        E += [(b, b + 1), (b + 2, b + 3)]
        ee.append((len(E) - 2, len(E) - 1))
    return (np.array(P0, np.float64).reshape(-1, 3), np.array(P1, np.float64).reshape(-1, 3),
            np.array(E, np.int32).reshape(-1, 2), np.array(F, np.int32).reshape(-1, 3),
            np.array(vf, np.int32).reshape(-1, 2), np.array(ee, np.int32).reshape(-1, 2))
