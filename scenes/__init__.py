"""Seeded synthetic scene generators.

These build the meshes and trajectories that both the CPU oracle and the
GPU path consume.  The module holds no part of the collision method's
arithmetic: it only produces vertex positions at t=0 and t=1 (float64,
row-major n x 3), edge lists (int32, n x 2, each undirected edge once with
the smaller vertex id first) and face lists (int32, n x 3).

The paper evaluates on simulated scenes (cloth, rigid bodies, large
elastic meshes; Section 3) that are not available here.  The generators
below stand in for them with the same kinds of structure: cloth
self-collision over a rigid obstacle, rigid-body contact between spheres,
and a large randomly perturbed closed surface.
"""
from .meshes import icosphere, grid_cloth, torus, edges_of_faces, merge_meshes
from .configs import (Scene, two_spheres, cloth_on_sphere, perturbed_torus, scene_batch, concat_scenes,
                      sample_pairs, degenerate_gadgets,
                      tiny_random_scene, sliding_slivers, make_config, CONFIG_NAMES)

__all__ = ["icosphere", "grid_cloth", "torus", "edges_of_faces", "merge_meshes",
           "Scene", "two_spheres", "cloth_on_sphere", "perturbed_torus",
           "tiny_random_scene", "sliding_slivers", "make_config", "CONFIG_NAMES"]
