"""Seeded scene generators: determinism, sizes and the CSR concatenation of batches (no GPU)."""
import numpy as np

import scenes
from scenes.meshes import edges_of_faces, icosphere


def test_edges_of_faces_matches_set_definition():
    V, F = icosphere(2)
    ref = sorted({tuple(sorted((int(f[i]), int(f[(i + 1) % 3])))) for f in F for i in range(3)})
    assert np.array_equal(edges_of_faces(F), np.array(ref, np.int32))
    # closed surface: Euler characteristic 2
    assert len(V) - len(ref) + len(F) == 2


def test_scene_batch_is_seeded_and_sized():
    a = scenes.scene_batch(seed=4, count=9, t_min=1e3, t_max=2e4)
    b = scenes.scene_batch(seed=4, count=9, t_min=1e3, t_max=2e4)
    assert [s.name for s in a] == ["cloth_on_sphere", "two_spheres", "perturbed_torus"] * 3
    for x, y in zip(a, b):
        assert np.array_equal(x.V0, y.V0) and np.array_equal(x.V1, y.V1) and np.array_equal(x.F, y.F)
        t = x.meta["target_tris"]
        assert 1e3 <= t <= 2e4
        # within a factor 2.5 of the target (icosphere levels step by 4)
        assert t / 2.5 <= x.nf <= 2.5 * t, (x.name, x.nf, t)


def test_concat_scenes_offsets_and_global_ids():
    scs = [scenes.tiny_random_scene(s, n_tris=2 + s) for s in range(4)]
    V0, V1, E, F, vo, eo, fo = scenes.concat_scenes(scs)
    assert list(vo) == list(np.cumsum([0] + [s.nv for s in scs]))
    assert list(eo) == list(np.cumsum([0] + [s.ne for s in scs]))
    assert list(fo) == list(np.cumsum([0] + [s.nf for s in scs]))
    for i, s in enumerate(scs):
        assert np.array_equal(V0[vo[i]:vo[i + 1]], s.V0)
        assert np.array_equal(F[fo[i]:fo[i + 1]] - vo[i], s.F)
        assert np.array_equal(E[eo[i]:eo[i + 1]] - vo[i], s.E)
        assert F[fo[i]:fo[i + 1]].min() >= vo[i] and F[fo[i]:fo[i + 1]].max() < vo[i + 1]


def test_sliding_slivers_is_seeded_and_long_on_one_axis():
    a, b = scenes.sliding_slivers(seed=3, n_tris=50), scenes.sliding_slivers(seed=3, n_tris=50)
    assert np.array_equal(a.V0, b.V0) and np.array_equal(a.V1, b.V1)
    assert a.nv == 150 and a.nf == 50 and a.ne == 150
    d = a.V1 - a.V0
    # each triangle slides rigidly along x only
    assert np.all(d[:, 1:] == 0.0)
    # (up to the rounding of V0 + shift)
    assert np.allclose(d[0::3, 0], d[1::3, 0], rtol=0, atol=1e-14) and np.allclose(d[0::3, 0], d[2::3, 0], rtol=0,
                                                                                     atol=1e-14)
