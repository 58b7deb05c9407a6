"""GPU narrow-phase options against the oracle, through the C ABI:

- Alg. 3's single shared t* (earliest_only): toi_min equals the per-pair mode's and the oracle's when the
  earliest pair did not reach the cap, and stays between the per-pair minimum and every uncapped pair's time
  otherwise;
- the minimum separation of Sec. 7 (per pair, or 0.2 d0 computed on the device) and the no-zero-TOI strategy of
  App. B: per-pair hit, TOI bits and n_enq identical to the oracle's;
- d0 (distance at t = 0) identical to the oracle's plain definition;
- App. B's step size (separation 0.2 d0, then no separation, no-zero strategy and 0.8 scaling when the first
  pass gives 0) identical to the oracle's composition;
- wide-stage pairs whose frontier outgrows its buffer resume from the level they saved (tiny buffers force it).
"""
import numpy as np
import pytest

import oracle
import scenes
from helpers import q24, scene_of_queries

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2112_06300_amd as ccd  # noqa: E402

DELTA = 1e-6
TRI = [(0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0)]


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ccd.Context(0)
    yield c
    c.close()


def dev(x, dt):
    return torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dt)


def scene_dev(s):
    return dev(s.V0, torch.float64), dev(s.V1, torch.float64), dev(s.E, torch.int32), dev(s.F, torch.int32)


def bits(x):
    return np.asarray(x, np.float64).view(np.int64)


def gpu_narrow(ctx, s, vf, ee, options=None, delta=DELTA, max_iter=10 ** 6):
    V0, V1, E, F = scene_dev(s)
    hit, toi, tmin, nenq = ctx.narrow(V0, V1, E, F, dev(vf, torch.int32), dev(ee, torch.int32), delta, max_iter,
                                      with_costs=True, options=options)
    torch.cuda.synchronize()
    return hit.cpu().numpy(), toi.cpu().numpy(), float(tmin.cpu()[0]), nenq.cpu().numpy()


def assert_same(g, o):
    gh, gt, gmin, gn = g
    oh, ot, on_, _, omin = o
    assert np.array_equal(gh, oh), np.nonzero(gh != oh)[0][:10]
    assert np.array_equal(bits(gt), bits(ot)), np.nonzero(bits(gt) != bits(ot))[0][:10]
    assert np.array_equal(gn, on_), np.nonzero(gn != on_)[0][:10]
    assert bits(gmin) == bits(omin)


def near_zero_scene():
    """Vertex-face and edge-edge pairs touching at t = 0, 1e-9 apart at t = 0, and crossing later, plus far
    pairs: the cases the no-zero strategy and the minimum separation change."""
    vq, eq = [], []
    for g in (0.0, 1e-9, 1e-6, 0.25):
        vq.append(q24([(0.25, 0.25, g)] + TRI, [(0.25, 0.25, g - 1.0)] + TRI))
        vq.append(q24([(0.3, 0.1, g)] + TRI, [(0.3, 0.6, g - 0.5)] + TRI))
        a0, a1, b0, b1 = (-1.0, 0.0, g), (1.0, 0.0, g), (0.0, -1.0, 0.0), (0.0, 1.0, 0.0)
        eq.append(q24([a0, a1, b0, b1], [(-1.0, 0.0, g - 1.0), (1.0, 0.0, g - 1.0), b0, b1]))
    vq.append(q24([(5.0, 5.0, 1.0)] + TRI, [(5.0, 5.0, -1.0)] + TRI))
    V0, V1, E, F, vf, ee = scene_of_queries(vq, eq)
    return scenes.Scene("near_zero", V0, V1, E, F), vf, ee


def cloth_pairs(n=48, seed=31):
    s = scenes.cloth_on_sphere(n=n, sphere_subdivisions=2, seed=seed)
    vf, ee = oracle.broad(s.V0, s.V1, s.E, s.F)
    return s, vf, ee


# --------------------------------------------------------------------------- d0
@pytest.mark.parametrize("make", [lambda: cloth_pairs(), lambda: near_zero_scene(),
                                  lambda: (lambda s: (s,) + tuple(oracle.all_pairs(s.E, s.F, s.nv)))(
                                      scenes.tiny_random_scene(11, n_tris=24, extent=1.0, motion=0.5))])
def test_initial_distance_matches_oracle(ctx, make):
    s, vf, ee = make()
    print(f"d0: {s.name} pairs={len(vf)}+{len(ee)}", flush=True)
    g = ctx.initial_distance(dev(s.V0, torch.float64), dev(s.E, torch.int32), dev(s.F, torch.int32),
                             dev(vf, torch.int32), dev(ee, torch.int32)).cpu().numpy()
    o = oracle.initial_distance(s.V0, s.E, s.F, vf, ee)
    assert np.array_equal(bits(g), bits(o)), np.nonzero(bits(g) != bits(o))[0][:10]


# --------------------------------------------------------------------------- minimum separation, no-zero
@pytest.mark.parametrize("make", [cloth_pairs, near_zero_scene])
@pytest.mark.parametrize("ms_kind", ["random", "d0"])
def test_min_separation_matches_oracle(ctx, make, ms_kind):
    s, vf, ee = make()
    n = len(vf) + len(ee)
    print(f"min separation ({ms_kind}): {s.name} pairs={n}", flush=True)
    if ms_kind == "random":
        rng = np.random.default_rng(n)
        ms = rng.uniform(0.0, 2e-3, n) * (rng.random(n) < 0.7)
        g = gpu_narrow(ctx, s, vf, ee, {"min_sep": dev(ms, torch.float64)})
    else:
        ms = 0.2 * oracle.initial_distance(s.V0, s.E, s.F, vf, ee)
        g = gpu_narrow(ctx, s, vf, ee, {"min_sep_d0_factor": 0.2})
    o = oracle.narrow(s.V0, s.V1, s.E, s.F, vf, ee, DELTA, 10 ** 6, ms=ms)
    assert_same(g, o)
    assert o[0].sum() >= gpu_narrow(ctx, s, vf, ee)[0].sum()  # a separation only adds hits


@pytest.mark.parametrize("make", [cloth_pairs, near_zero_scene])
@pytest.mark.parametrize("max_iter", [10, 10 ** 6])
def test_no_zero_matches_oracle(ctx, make, max_iter):
    s, vf, ee = make()
    print(f"no-zero: {s.name} pairs={len(vf)}+{len(ee)} max_iter={max_iter}", flush=True)
    g = gpu_narrow(ctx, s, vf, ee, {"no_zero_toi": 1}, max_iter=max_iter)
    o = oracle.narrow(s.V0, s.V1, s.E, s.F, vf, ee, DELTA, max_iter, no_zero=True)
    assert_same(g, o)


def test_min_separation_rejects_bad_values(ctx):
    s, vf, ee = near_zero_scene()
    n = len(vf) + len(ee)
    for bad in (-1e-3, float("nan"), float("inf")):
        ms = np.zeros(n)
        ms[3] = bad
        with pytest.raises(ccd.CCDError):
            gpu_narrow(ctx, s, vf, ee, {"min_sep": dev(ms, torch.float64)})
    with pytest.raises(ccd.CCDError):
        gpu_narrow(ctx, s, vf, ee, {"min_sep_d0_factor": -0.5})
    with pytest.raises(ccd.CCDError):
        gpu_narrow(ctx, s, vf, ee, {"min_sep": dev(np.zeros(n), torch.float64), "min_sep_d0_factor": 0.2})


# --------------------------------------------------------------------------- Alg. 3's shared t*
def check_earliest(ctx, s, vf, ee, max_iter=10 ** 6, options=None):
    gh, gt, gmin, gn = gpu_narrow(ctx, s, vf, ee, options, max_iter=max_iter)
    opt = dict(options or {})
    ms = opt.pop("min_sep", None)
    g_glob = gpu_narrow(ctx, s, vf, ee, dict(opt, earliest_only=1, **({"min_sep": ms} if ms is not None else {})),
                        max_iter=max_iter)[2]
    oh, ot, on_, _, omin = oracle.narrow(s.V0, s.V1, s.E, s.F, vf, ee, DELTA, max_iter,
                                         ms=None if ms is None else ms.cpu().numpy(),
                                         no_zero=bool(opt.get("no_zero_toi")))
    assert bits(gmin) == bits(omin)
    capped = on_ > max_iter
    if not np.any(capped & (ot == omin)):
        # the earliest pair did not reach the cap: Alg. 3's t* is the per-pair minimum exactly
        assert bits(g_glob) == bits(omin), (g_glob, omin)
        og, _ = oracle.narrow_global(s.V0, s.V1, s.E, s.F, vf, ee, DELTA, max_iter,
                                     ms=None if ms is None else ms.cpu().numpy(),
                                     no_zero=bool(opt.get("no_zero_toi")))
        assert bits(og) == bits(omin)
    else:
        free = ot[~capped]
        assert omin <= g_glob <= (free.min() if len(free) else np.inf)
    return g_glob, omin


@pytest.mark.parametrize("make", [lambda: cloth_pairs(64, 5), near_zero_scene,
                                  lambda: (lambda s: (s,) + tuple(oracle.broad(s.V0, s.V1, s.E, s.F)))(
                                      scenes.two_spheres())])
def test_earliest_only_matches_per_pair_minimum(ctx, make):
    s, vf, ee = make()
    print(f"earliest only: {s.name} pairs={len(vf)}+{len(ee)}", flush=True)
    check_earliest(ctx, s, vf, ee)


def test_earliest_only_two_spheres_all_pairs(ctx):
    """Every VF and EE pair of the two spheres (10.6M queries, most far apart)."""
    s = scenes.two_spheres()
    vf, ee = oracle.all_pairs(s.E, s.F, s.nv)
    print(f"earliest only: all pairs of two spheres {len(vf)}+{len(ee)}", flush=True)
    g, o = check_earliest(ctx, s, vf, ee)
    assert 0.0 < o < 1.0


def test_earliest_only_with_capped_pairs(ctx):
    """Degenerate sliding pairs at max_iter 1e3 and 1e6: capped pairs never push the shared t* below the
    per-pair minimum or above an uncapped pair's time; with no-zero and separations too."""
    from test_gpu_parity import _degenerate_scene
    s = _degenerate_scene()
    vf, ee = oracle.all_pairs(s.E, s.F, s.nv)
    for max_iter in (1000, 10 ** 6):
        check_earliest(ctx, s, vf, ee, max_iter=max_iter)
    check_earliest(ctx, s, vf, ee, max_iter=1000, options={"no_zero_toi": 1})
    ms = dev(np.full(len(vf) + len(ee), 1e-4), torch.float64)
    check_earliest(ctx, s, vf, ee, max_iter=1000, options={"min_sep": ms})


# --------------------------------------------------------------------------- App. B step
def oracle_step(s, ms_factor=0.2, scale=0.8):
    vf, ee = oracle.broad(s.V0, s.V1, s.E, s.F)
    ms = ms_factor * oracle.initial_distance(s.V0, s.E, s.F, vf, ee)
    t = oracle.narrow(s.V0, s.V1, s.E, s.F, vf, ee, DELTA, 10 ** 6, ms=ms)[4]
    if t == 0.0:
        return oracle.narrow(s.V0, s.V1, s.E, s.F, vf, ee, DELTA, 10 ** 6, no_zero=True)[4] * scale, True
    return t, False


def touching_cloth():
    """The small cloth with one of its vertices placed on the sphere at t = 0 (a pair touching at t = 0)."""
    s = scenes.cloth_on_sphere(n=24, sphere_subdivisions=2, seed=8)
    V0, V1 = s.V0.copy(), s.V1.copy()
    nc = 24 * 24
    # the sphere's first vertex coincides with a cloth vertex at t = 0 and moves away
    V0[nc] = V0[0]
    V1[nc] = V0[0] + (0.0, -0.5, 0.0)
    return scenes.Scene("touching_cloth", V0, V1, s.E, s.F)


@pytest.mark.parametrize("make", [lambda: scenes.cloth_on_sphere(n=48, sphere_subdivisions=2, seed=9),
                                  touching_cloth, scenes.two_spheres])
def test_toi_step_matches_oracle(ctx, make):
    s = make()
    print(f"toi step: {s.name}", flush=True)
    V0, V1, E, F = scene_dev(s)
    vf = torch.empty((8 * s.nb, 2), dtype=torch.int32, device="cuda")
    ee = torch.empty((8 * s.nb, 2), dtype=torch.int32, device="cuda")
    t, rerun, n_vf, n_ee = ctx.toi_step(V0, V1, E, F, vf, ee)
    ot, orerun = oracle_step(s)
    assert rerun == orerun
    assert bits(t) == bits(ot), (t, ot)


# --------------------------------------------------------------------------- resume of overflowing frontiers
@pytest.mark.parametrize("tuning", [{"heavy_cap_log2": 8, "heavy_slots": 16},
                                    {"heavy_cap_log2": 9, "heavy_block": 256, "heavy_lds": 0}])
def test_overflowing_frontiers_resume(ctx, tuning):
    """Tiny wide-stage buffers: most wide-stage pairs outgrow them, save their level and resume from it; every
    per-pair result stays identical to the oracle's."""
    from test_gpu_parity import _degenerate_scene
    ctx.set_tuning(tuning)
    try:
        s = _degenerate_scene()
        vf, ee = oracle.all_pairs(s.E, s.F, s.nv)
        for max_iter in (1000, 10 ** 6):
            g = gpu_narrow(ctx, s, vf, ee, max_iter=max_iter)
            if max_iter > 10 * (1 << tuning["heavy_cap_log2"]):
                assert ctx.stats()["heavy_reruns"] > 0  # frontiers far above the buffers' size
            assert_same(g, oracle.narrow(s.V0, s.V1, s.E, s.F, vf, ee, DELTA, max_iter))
    finally:
        ctx.set_tuning(None)
