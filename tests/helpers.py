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
