"""Closed-form mesh builders (float64 vertices, int32 topology)."""
import numpy as np


def edges_of_faces(F):
    """Unique undirected edges of a triangle list, each as (min, max), sorted."""
    F = np.asarray(F, dtype=np.int64)
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], axis=0)
    e.sort(axis=1)
    return _unique_rows(e)[0].astype(np.int32)


def _unique_rows(e):
    """np.unique(e, axis=0, return_inverse=True) for non-negative (n, 2) int64 rows, via 1-D keys."""
    if len(e) == 0:
        return e.reshape(0, 2), np.zeros(0, np.int64)
    m = int(e.max()) + 1
    keys, inv = np.unique(e[:, 0] * m + e[:, 1], return_inverse=True)
    return np.stack([keys // m, keys % m], 1), inv.reshape(-1)


def icosphere(subdivisions, radius=1.0, center=(0.0, 0.0, 0.0)):
    """Icosahedron subdivided `subdivisions` times and projected on a sphere.

    Vertex count 10*4^k + 2, face count 20*4^k.
    """
    p = (1.0 + 5.0 ** 0.5) / 2.0
    V = [(-1, p, 0), (1, p, 0), (-1, -p, 0), (1, -p, 0),
         (0, -1, p), (0, 1, p), (0, -1, -p), (0, 1, -p),
         (p, 0, -1), (p, 0, 1), (-p, 0, -1), (-p, 0, 1)]
    F = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    V = np.array(V, dtype=np.float64)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    F = np.array(F, dtype=np.int64)
    for _ in range(subdivisions):
        e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], axis=0)
        e.sort(axis=1)
        uniq, inv = _unique_rows(e)
        mids = V[uniq[:, 0]] + V[uniq[:, 1]]
        mids /= np.linalg.norm(mids, axis=1, keepdims=True)
        base = len(V)
        V = np.concatenate([V, mids], axis=0)
        nf = len(F)
        m01 = base + inv[0:nf]
        m12 = base + inv[nf:2 * nf]
        m20 = base + inv[2 * nf:3 * nf]
        a, b, c = F[:, 0], F[:, 1], F[:, 2]
        F = np.concatenate([np.stack([a, m01, m20], 1), np.stack([b, m12, m01], 1),
                            np.stack([c, m20, m12], 1), np.stack([m01, m12, m20], 1)], axis=0)
    V = V * radius + np.asarray(center, dtype=np.float64)
    return V, F.astype(np.int32)


def grid_cloth(n, side, height, axis_normal=1):
    """n x n vertex grid of the given side length in the plane coord[axis_normal]=height.

    One diagonal per quad: 2 (n-1)^2 faces, 2 n (n-1) + (n-1)^2 edges.
    """
    s = np.linspace(-side / 2.0, side / 2.0, n)
    a, b = np.meshgrid(s, s, indexing="ij")
    V = np.zeros((n * n, 3), dtype=np.float64)
    other = [k for k in range(3) if k != axis_normal]
    V[:, other[0]] = a.reshape(-1)
    V[:, other[1]] = b.reshape(-1)
    V[:, axis_normal] = height
    idx = np.arange(n * n).reshape(n, n)
    i00 = idx[:-1, :-1].reshape(-1)
    i10 = idx[1:, :-1].reshape(-1)
    i01 = idx[:-1, 1:].reshape(-1)
    i11 = idx[1:, 1:].reshape(-1)
    F = np.concatenate([np.stack([i00, i10, i11], 1), np.stack([i00, i11, i01], 1)], axis=0)
    return V, F.astype(np.int32)


def torus(n_major, n_minor, R=1.0, r=0.4):
    """Closed torus grid: n_major*n_minor vertices, 2*n_major*n_minor faces."""
    th = 2.0 * np.pi * np.arange(n_major) / n_major
    ph = 2.0 * np.pi * np.arange(n_minor) / n_minor
    T, P = np.meshgrid(th, ph, indexing="ij")
    V = np.stack([(R + r * np.cos(P)) * np.cos(T), (R + r * np.cos(P)) * np.sin(T), r * np.sin(P)], -1)
    V = V.reshape(-1, 3).astype(np.float64)
    i = np.arange(n_major)
    j = np.arange(n_minor)
    I, J = np.meshgrid(i, j, indexing="ij")
    I1 = (I + 1) % n_major
    J1 = (J + 1) % n_minor
    a = (I * n_minor + J).reshape(-1)
    b = (I1 * n_minor + J).reshape(-1)
    c = (I1 * n_minor + J1).reshape(-1)
    d = (I * n_minor + J1).reshape(-1)
    F = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)], axis=0)
    return V, F.astype(np.int32)


def merge_meshes(parts):
    """Concatenate (V0, V1, F) triples into one mesh, offsetting face indices."""
    V0s, V1s, Fs = [], [], []
    off = 0
    for V0, V1, F in parts:
        V0s.append(V0)
        V1s.append(V1)
        Fs.append(np.asarray(F, dtype=np.int64) + off)
        off += len(V0)
    return (np.concatenate(V0s).astype(np.float64), np.concatenate(V1s).astype(np.float64),
            np.concatenate(Fs).astype(np.int32))
