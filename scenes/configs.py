"""The benchmark workloads as seeded synthetic scenes.

Each generator uses numpy's PCG64 with a fixed default seed and returns a
`Scene`.  Geometry constants that the workload descriptions leave open
(sphere placement, cloth height, torus radii, ...) are fixed here once.
"""
from dataclasses import dataclass, field

import numpy as np

from .meshes import icosphere, grid_cloth, torus, edges_of_faces, merge_meshes


@dataclass
class Scene:
    name: str
    V0: np.ndarray          # (nv, 3) float64, positions at t=0
    V1: np.ndarray          # (nv, 3) float64, positions at t=1
    E: np.ndarray           # (ne, 2) int32, e[0] < e[1]
    F: np.ndarray           # (nf, 3) int32
    meta: dict = field(default_factory=dict)

    @property
    def nv(self):
        return int(self.V0.shape[0])

    @property
    def ne(self):
        return int(self.E.shape[0])

    @property
    def nf(self):
        return int(self.F.shape[0])

    @property
    def nb(self):
        return self.nv + self.ne + self.nf


def _scene(name, V0, V1, F, **meta):
    V0 = np.ascontiguousarray(V0, dtype=np.float64)
    V1 = np.ascontiguousarray(V1, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.int32)
    E = np.ascontiguousarray(edges_of_faces(F), dtype=np.int32)
    return Scene(name, V0, V1, E, F, dict(meta))


def two_spheres(seed=1, subdivisions=3, jitter=1e-3, gap=0.05, displacement=0.1):
    """Two unit icospheres approaching each other along x.

    Centres at (-(1+gap/2), 0, 0) and (+(1+gap/2), 0, 0); every vertex gets
    the same N(0, jitter^2) offset at t=0 and t=1; each sphere moves
    `displacement` toward the other, so first contact is near t = gap/(2*displacement).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    c = 1.0 + gap / 2.0
    parts = []
    for sgn in (-1.0, 1.0):
        V, F = icosphere(subdivisions, 1.0, (sgn * c, 0.0, 0.0))
        V = V + rng.normal(0.0, jitter, size=V.shape)
        V1 = V.copy()
        V1[:, 0] -= sgn * displacement
        parts.append((V, V1, F))
    V0, V1, F = merge_meshes(parts)
    return _scene("two_spheres", V0, V1, F, seed=seed, subdivisions=subdivisions)


def cloth_on_sphere(seed=2, n=256, side=3.0, sphere_subdivisions=5, noise=0.3, drop=0.5):
    """n x n cloth falling onto a static unit icosphere at the origin.

    The cloth lies flat in the plane y = 1 + 0.25*e (e = mean cloth edge
    length) at t=0; at t=1 every cloth vertex has moved by
    N(0, (noise*e)^2) per coordinate plus (0, -drop*e, 0).  The union of the
    two meshes yields cloth self pairs and cloth-sphere pairs.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    Vc, Fc = grid_cloth(n, side, 0.0, axis_normal=1)
    Ec = edges_of_faces(Fc)
    elen = np.linalg.norm(Vc[Ec[:, 0]] - Vc[Ec[:, 1]], axis=1)
    ebar = float(elen.mean())
    Vc[:, 1] = 1.0 + 0.25 * ebar
    Vc1 = Vc + rng.normal(0.0, noise * ebar, size=Vc.shape)
    Vc1[:, 1] -= drop * ebar
    Vs, Fs = icosphere(sphere_subdivisions, 1.0)
    V0, V1, F = merge_meshes([(Vc, Vc1, Fc), (Vs, Vs.copy(), Fs)])
    return _scene("cloth_on_sphere", V0, V1, F, seed=seed, n=n, mean_edge=ebar)


def perturbed_torus(seed=3, n_major=1000, n_minor=500, R=1.0, r=0.4, rest_noise=0.1, noise=0.5, gadgets=0):
    """Closed torus surface with Gaussian vertex perturbations.

    t=0 positions are the torus plus N(0, (rest_noise*e)^2), t=1 positions add
    N(0, (noise*e)^2) per coordinate (e = mean edge length of the clean torus).
    With gadgets > 0, that many near-degenerate two-triangle gadgets
    (`degenerate_gadgets`) are placed inside the tube, where they pair only
    with each other.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    V, F = torus(n_major, n_minor, R, r)
    E = edges_of_faces(F)
    ebar = float(np.linalg.norm(V[E[:, 0]] - V[E[:, 1]], axis=1).mean())
    V0 = V + rng.normal(0.0, rest_noise * ebar, size=V.shape)
    V1 = V0 + rng.normal(0.0, noise * ebar, size=V.shape)
    if gadgets > 0:
        G0, G1, GF = degenerate_gadgets(rng, gadgets, ebar, R=R, tube=0.6 * r)
        V0, V1, F = merge_meshes([(V0, V1, F), (G0, G1, GF)])
    return _scene("perturbed_torus", V0, V1, F, seed=seed, mean_edge=ebar, gadgets=int(gadgets))


# Gadget kinds: (pair type, path, separation / height in units of the mean edge)
GADGET_KINDS = [("ee", "parallel", 0.0), ("vf", "interior", 0.0), ("ee", "parallel", 1e-12),
                ("vf", "edge", 0.0), ("ee", "parallel", 1e-9), ("vf", "vertex", 0.0),
                ("vf", "interior", 1e-12), ("vf", "edge", 1e-9), ("vf", "vertex", 1e-12)]


def degenerate_gadgets(rng, count, ebar, R=1.0, tube=0.24):
    """`count` two-triangle gadgets with near-degenerate contacts, inside a torus tube.

    Every gadget is axis-aligned with dyadic coordinates (exactly representable,
    so zero separations are exact) and sits on its own lattice cell within
    distance `tube` of the circle of radius R in the z = 0 plane:
      ee: a static triangle with an edge along x, and a triangle whose edge is
          parallel to it at separation s (0, 1e-12 e or 1e-9 e) sliding along it;
      vf: a static triangle in the plane z = 0 and a triangle whose lowest
          vertex moves parallel to that plane at height s, through the face's
          interior, along one of its edges, or through one of its vertices.
    Returns (V0, V1, F) of all gadgets.
    """
    q = 2.0 ** -12
    L, w = 2.0 ** -7, 2.0 ** -8          # edge length and triangle width
    spacing = 4.0 * L
    # lattice points inside the tube, in a seeded random order
    n_ring = int(2.0 * np.pi * R / spacing)
    k = int(tube / spacing)
    pts = []
    for i in range(n_ring):
        th = 2.0 * np.pi * i / n_ring
        for a in range(-k, k + 1):
            for b in range(-k, k + 1):
                if (a * a + b * b) * spacing * spacing <= tube * tube:
                    rho = R + a * spacing
                    pts.append((rho * np.cos(th), rho * np.sin(th), b * spacing))
    pts = np.array(pts)
    if count > len(pts):
        raise ValueError(f"at most {len(pts)} gadgets fit in the tube")
    pts = pts[rng.permutation(len(pts))[:count]]
    pts = np.round(pts / q) * q
    V0s, V1s, Fs = [], [], []
    for g, c in enumerate(pts):
        kind, path, sep = GADGET_KINDS[g % len(GADGET_KINDS)]
        s = sep * ebar
        if kind == "ee":
            a = [(0, 0, 0), (L, 0, 0), (0, -w, 0)]
            b = [(-L / 2, 0, s), (L / 2, 0, s), (-L / 2, 0, s + w)]
            a1 = a
            b1 = [(x + L, y, z) for x, y, z in b]   # slides along the static edge
        else:
            a = [(0, 0, 0), (L, 0, 0), (0, L, 0)]
            a1 = a
            if path == "interior":
                p0, p1 = (-L / 4, L / 4, s), (L, L / 4, s)
            elif path == "edge":
                p0, p1 = (-L / 4, 0, s), (L + L / 4, 0, s)
            else:
                p0, p1 = (-L / 4, -L / 4, s), (L / 4, L / 4, s)
            b = [p0, (p0[0] + w, p0[1], p0[2] + w), (p0[0], p0[1] + w, p0[2] + w)]
            d = np.subtract(p1, p0)
            b1 = [tuple(np.add(v, d)) for v in b]
        base = 6 * g
        V0s.append(np.array(a + b, np.float64) + c)
        V1s.append(np.array(a1 + b1, np.float64) + c)
        Fs.append(np.array([[base, base + 1, base + 2], [base + 3, base + 4, base + 5]], np.int64))
    if count == 0:
        return np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 3), np.int32)
    return np.concatenate(V0s), np.concatenate(V1s), np.concatenate(Fs).astype(np.int32)


def tiny_random_scene(seed, n_tris=6, extent=1.0, motion=0.6, dyadic_bits=None):
    """A few disconnected triangles with random linear motion, for exhaustive checks.

    With `dyadic_bits=b` every coordinate is a multiple of 2^-b, so exact
    rational arithmetic on the inputs is cheap.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    V0 = rng.uniform(-extent, extent, size=(3 * n_tris, 3))
    V1 = V0 + rng.uniform(-motion, motion, size=V0.shape)
    if dyadic_bits is not None:
        q = float(2 ** dyadic_bits)
        V0 = np.round(V0 * q) / q
        V1 = np.round(V1 * q) / q
    F = np.arange(3 * n_tris, dtype=np.int32).reshape(n_tris, 3)
    return _scene("tiny_random", V0, V1, F, seed=seed)


def sliding_slivers(seed=3, n_tris=4000, length=20.0, size=0.01, slide=5.0):
    """Small disconnected triangles scattered along a long bar, each sliding
    along it by up to +-slide: boxes are long on the sweep axis and tiny on the
    other two, so sweep windows hold hundreds to thousands of candidates while
    few of them overlap (a stress case for long windows).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    c = np.column_stack([rng.uniform(-length / 2, length / 2, n_tris), rng.uniform(-1.0, 1.0, (n_tris, 2))])
    V0 = np.repeat(c, 3, axis=0) + rng.uniform(-size, size, (3 * n_tris, 3))
    shift = np.zeros((n_tris, 3))
    shift[:, 0] = rng.uniform(-slide, slide, n_tris)
    V1 = V0 + np.repeat(shift, 3, axis=0)
    F = np.arange(3 * n_tris, dtype=np.int32).reshape(n_tris, 3)
    return _scene("sliding_slivers", V0, V1, F, seed=seed)


def scene_batch(seed=4, count=64, t_min=1e3, t_max=2e5):
    """`count` scenes with log-uniform triangle counts in [t_min, t_max].

    Types cycle cloth-on-sphere, two spheres, perturbed torus; scene i uses
    seed 1000 + i and the resolution whose triangle count is nearest to its
    target (icosphere levels only come in powers of 4).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    targets = np.round(np.exp(rng.uniform(np.log(t_min), np.log(t_max), count))).astype(np.int64)
    out = []
    for i, t in enumerate(targets):
        s = 1000 + i
        if i % 3 == 0:
            k = int(np.clip(np.round(np.log(max(t / 4.0, 20.0) / 20.0) / np.log(4.0)), 0, 5))
            cloth = max(int(t) - 20 * 4 ** k, 8)
            n = int(round(np.sqrt(cloth / 2.0))) + 1
            out.append(cloth_on_sphere(seed=s, n=n, sphere_subdivisions=k))
        elif i % 3 == 1:
            k = int(np.clip(np.round(np.log(t / 40.0) / np.log(4.0)), 0, 6))
            out.append(two_spheres(seed=s, subdivisions=k))
        else:
            nm = max(3, int(round(np.sqrt(t / 4.0))))
            out.append(perturbed_torus(seed=s, n_major=2 * nm, n_minor=nm))
        out[-1].meta["target_tris"] = int(t)
    return out


def concat_scenes(scenes):
    """Concatenate scenes in CSR layout: (V0, V1, E, F, v_off, e_off, f_off), vertex ids global."""
    v_off = np.zeros(len(scenes) + 1, np.int64)
    e_off = np.zeros(len(scenes) + 1, np.int64)
    f_off = np.zeros(len(scenes) + 1, np.int64)
    for i, s in enumerate(scenes):
        v_off[i + 1] = v_off[i] + s.nv
        e_off[i + 1] = e_off[i] + s.ne
        f_off[i + 1] = f_off[i] + s.nf
    V0 = np.concatenate([s.V0 for s in scenes]) if scenes else np.zeros((0, 3))
    V1 = np.concatenate([s.V1 for s in scenes]) if scenes else np.zeros((0, 3))
    E = np.concatenate([s.E + v_off[i] for i, s in enumerate(scenes)]).astype(np.int32)
    F = np.concatenate([s.F + v_off[i] for i, s in enumerate(scenes)]).astype(np.int32)
    return V0, V1, E, F, v_off, e_off, f_off


def sample_pairs(vf, ee, count, seed=5):
    """`count` candidate pairs drawn with replacement from the candidates (vf, ee) of a scene.

    The candidates are put in canonical (sorted) order first, so the draw does
    not depend on the order a broad phase emitted them in; the VF / EE mix and
    every other property of the candidate distribution (the degenerate share
    among them) is kept in expectation.  Returns (vf_sample, ee_sample).
    """
    vf = np.asarray(vf, np.int32).reshape(-1, 2)
    ee = np.asarray(ee, np.int32).reshape(-1, 2)
    vf = vf[np.lexsort((vf[:, 1], vf[:, 0]))]
    ee = ee[np.lexsort((ee[:, 1], ee[:, 0]))]
    rng = np.random.Generator(np.random.PCG64(seed))
    pick = rng.integers(0, len(vf) + len(ee), size=count)
    pick.sort()
    nvf = int(np.searchsorted(pick, len(vf)))
    return vf[pick[:nvf]], ee[pick[nvf:] - len(vf)]


CONFIG_NAMES = {1: "two_spheres", 2: "cloth_on_sphere", 3: "perturbed_torus"}


def make_config(k, **kw):
    """Scene for workload k (1: two spheres, 2: cloth on sphere, 3: perturbed torus)."""
    if k == 1:
        return two_spheres(**kw)
    if k == 2:
        return cloth_on_sphere(**kw)
    if k == 3:
        return perturbed_torus(**kw)
    raise ValueError(f"no scene generator for workload {k}")
