"""GPU path (through the C ABI) against the CPU oracle, element by element.

Candidate sets must be identical; per-pair hit flags, times of impact (bit
patterns) and enqueue counts must be identical; the global minimum must be
identical.  All inputs are seeded synthetic scenes.
"""
import numpy as np
import pytest

import oracle
import scenes
from helpers import q24, deep_split_query, scene_of_queries

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2112_06300_amd as ccd  # noqa: E402

DELTA = 1e-6


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ccd.Context(0)
    yield c
    c.close()


def canon(p):
    p = np.asarray(p).reshape(-1, 2)
    if len(p) == 0:
        return p
    o = np.lexsort((p[:, 1], p[:, 0]))
    return p[o]


def dev(x, dt):
    return torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dt)


def run_broad(ctx, s, **kw):
    vf, ee = ctx.broad(dev(s.V0, torch.float64), dev(s.V1, torch.float64), dev(s.E, torch.int32),
                       dev(s.F, torch.int32), **kw)
    return canon(vf.cpu().numpy()), canon(ee.cpu().numpy())


def check_broad(ctx, s):
    print(f"broad parity: {s.name} nv={s.nv} ne={s.ne} nf={s.nf}", flush=True)
    gvf, gee = run_broad(ctx, s)
    ovf, oee = oracle.broad(s.V0, s.V1, s.E, s.F)
    assert np.array_equal(gvf, ovf), (len(gvf), len(ovf))
    assert np.array_equal(gee, oee), (len(gee), len(oee))
    return ovf, oee


def run_narrow(ctx, s, vf, ee, delta=DELTA, max_iter=10 ** 6):
    hit, toi, tmin, nenq = ctx.narrow(dev(s.V0, torch.float64), dev(s.V1, torch.float64), dev(s.E, torch.int32),
                                      dev(s.F, torch.int32), dev(vf, torch.int32), dev(ee, torch.int32),
                                      delta, max_iter, with_costs=True)
    torch.cuda.synchronize()
    return hit.cpu().numpy(), toi.cpu().numpy(), float(tmin.cpu()[0]), nenq.cpu().numpy()


def check_narrow(ctx, s, vf, ee, delta=DELTA, max_iter=10 ** 6):
    print(f"narrow parity: {s.name} pairs={len(vf)}+{len(ee)} delta={delta} max_iter={max_iter}", flush=True)
    gh, gt, gmin, gn = run_narrow(ctx, s, vf, ee, delta, max_iter)
    oh, ot, on_, _, omin = oracle.narrow(s.V0, s.V1, s.E, s.F, vf, ee, delta, max_iter)
    assert np.array_equal(gh, oh), np.nonzero(gh != oh)[0][:10]
    assert np.array_equal(gt.view(np.int64), ot.view(np.int64)), np.nonzero(gt != ot)[0][:10]
    assert np.array_equal(gn, on_), np.nonzero(gn != on_)[0][:10]
    assert np.float64(gmin).view(np.int64) == np.float64(omin).view(np.int64)
    return oh, ot, on_


# --------------------------------------------------------------------------- broad
def test_broad_two_spheres(ctx):
    check_broad(ctx, scenes.two_spheres())


def test_broad_cloth_on_sphere_full(ctx):
    s = scenes.cloth_on_sphere()
    vf, ee = check_broad(ctx, s)
    assert len(vf) > 100000 and len(ee) > 400000


@pytest.mark.parametrize("n,sub", [(2, 0), (3, 1), (17, 2), (65, 3)])
def test_broad_ragged_cloth(ctx, n, sub):
    check_broad(ctx, scenes.cloth_on_sphere(n=n, sphere_subdivisions=sub, seed=100 + n))


@pytest.mark.parametrize("seed", range(4))
def test_broad_tiny_random(ctx, seed):
    check_broad(ctx, scenes.tiny_random_scene(seed, n_tris=30 + 37 * seed, extent=1.0, motion=0.5,
                                              dyadic_bits=(3 if seed % 2 else None)))


def test_broad_long_windows(ctx):
    """Sweep windows of up to ~1,000 (vertex-face) and ~3,200 (edge-edge) candidates: several chunks per tile."""
    s = scenes.sliding_slivers()
    vf, ee = check_broad(ctx, s)
    assert len(vf) > 0 and len(ee) > 0
    check_narrow(ctx, s, vf, ee)


def test_broad_extreme_coordinates(ctx):
    rng = np.random.default_rng(5)
    s = scenes.tiny_random_scene(9, n_tris=60, extent=1.0, motion=0.5)
    scale = 2.0 ** rng.integers(-140, 100, size=(s.nv, 1))  # float32 subnormal range to huge
    s.V0 = np.ascontiguousarray(s.V0 * scale)
    s.V1 = np.ascontiguousarray(s.V1 * scale)
    s.V0[::7] = -0.0
    check_broad(ctx, s)


def test_broad_identical_boxes(ctx):
    s = scenes.tiny_random_scene(1, n_tris=12)
    s.V0[:] = 0.5
    s.V1[:] = 0.5
    vf, ee = check_broad(ctx, s)
    assert len(vf) == s.nv * s.nf - 3 * s.nf


def test_broad_empty_and_partial(ctx):
    s = scenes.tiny_random_scene(2, n_tris=5)
    for nv, E, F in [(0, np.zeros((0, 2), np.int32), np.zeros((0, 3), np.int32)),
                     (s.nv, np.zeros((0, 2), np.int32), np.zeros((0, 3), np.int32)),
                     (s.nv, s.E, np.zeros((0, 3), np.int32)),
                     (s.nv, np.zeros((0, 2), np.int32), s.F)]:
        t = scenes.Scene("partial", s.V0[:nv], s.V1[:nv], E, F)
        check_broad(ctx, t)


def test_broad_capacity_error(ctx):
    s = scenes.two_spheres()
    ovf, oee = oracle.broad(s.V0, s.V1, s.E, s.F)
    V0, V1 = dev(s.V0, torch.float64), dev(s.V1, torch.float64)
    E, F = dev(s.E, torch.int32), dev(s.F, torch.int32)
    vf = torch.empty((10, 2), dtype=torch.int32, device="cuda")
    ee = torch.empty((len(oee), 2), dtype=torch.int32, device="cuda")
    with pytest.raises(ccd.CCDError) as ei:
        ctx.broad_into(V0, V1, E, F, vf, ee)
    assert ei.value.status == ccd.CCD_ERR_CAPACITY
    # automatic resizing path
    gvf, gee = run_broad(ctx, s, vf_cap=10, ee_cap=10)
    assert np.array_equal(gvf, ovf) and np.array_equal(gee, oee)


def test_broad_rejects_bad_input(ctx):
    s = scenes.tiny_random_scene(2, n_tris=5)
    F = s.F.copy()
    F[1, 2] = s.nv
    with pytest.raises(ccd.CCDError) as ei:
        run_broad(ctx, scenes.Scene("bad", s.V0, s.V1, s.E, F))
    assert ei.value.status == ccd.CCD_ERR_INVALID_ARG
    V0 = s.V0.copy()
    V0[3, 1] = np.nan
    with pytest.raises(ccd.CCDError) as ei:
        run_broad(ctx, scenes.Scene("nan", V0, s.V1, s.E, s.F))
    assert ei.value.status == ccd.CCD_ERR_NONFINITE


@pytest.mark.parametrize("classes", [1, 2, 3, 4, 8])
def test_broad_query_classes(ctx, classes):
    """The sweep's queries grouped into extent classes before they are cut into tiles (tiles then walk
    different candidate ranges): the pair set never changes.  Mixed extents (long slivers), a full-size
    cloth, ragged tails, empty segments and one lone box."""
    print(f"sweep_classes {classes}", flush=True)
    ctx.set_tuning({"sweep_classes": classes})
    try:
        check_broad(ctx, scenes.sliding_slivers())
        check_broad(ctx, scenes.cloth_on_sphere(n=96, sphere_subdivisions=3, seed=21))
        check_broad(ctx, scenes.cloth_on_sphere(n=17, sphere_subdivisions=2, seed=117))
        check_broad(ctx, scenes.tiny_random_scene(3, n_tris=67, extent=1.0, motion=0.5))
        t = scenes.tiny_random_scene(2, n_tris=5)
        for nv, E, F in [(0, np.zeros((0, 2), np.int32), np.zeros((0, 3), np.int32)),
                         (1, np.zeros((0, 2), np.int32), np.zeros((0, 3), np.int32)),
                         (t.nv, t.E, np.zeros((0, 3), np.int32)),
                         (t.nv, np.zeros((0, 2), np.int32), t.F)]:
            check_broad(ctx, scenes.Scene("partial", t.V0[:nv], t.V1[:nv], E, F))
    finally:
        ctx.set_tuning(None)


# --------------------------------------------------------------------------- narrow
def test_narrow_two_spheres_candidates(ctx):
    s = scenes.two_spheres()
    vf, ee = oracle.broad(s.V0, s.V1, s.E, s.F)
    check_narrow(ctx, s, vf, ee)


def test_narrow_two_spheres_all_pairs(ctx):
    s = scenes.two_spheres()
    vf, ee = oracle.all_pairs(s.E, s.F, s.nv)
    assert len(vf) + len(ee) == 10631100
    oh, ot, _ = check_narrow(ctx, s, vf, ee)
    assert oh.sum() > 0


def test_narrow_cloth_on_sphere_full(ctx):
    s = scenes.cloth_on_sphere()
    vf, ee = oracle.broad(s.V0, s.V1, s.E, s.F)
    check_narrow(ctx, s, vf, ee)


@pytest.mark.parametrize("seed", range(3))
def test_narrow_tiny_all_pairs(ctx, seed):
    s = scenes.tiny_random_scene(seed, n_tris=6, extent=0.5, motion=1.0, dyadic_bits=(4 if seed else None))
    vf, ee = oracle.all_pairs(s.E, s.F, s.nv)
    check_narrow(ctx, s, vf, ee)


@pytest.mark.parametrize("delta", [1e-2, 1e-4, 1e-8, 1e-12])
def test_narrow_delta_sweep(ctx, delta):
    s = scenes.two_spheres()
    vf, ee = oracle.broad(s.V0, s.V1, s.E, s.F)
    check_narrow(ctx, s, vf[::3], ee[::3], delta=delta)


def _degenerate_scene():
    """Parallel edges sliding onto each other and grazing vertex-face pairs (wide frontiers)."""
    pts0, pts1, faces, edges = [], [], [], []

    def add(p0, p1):
        pts0.append(p0)
        pts1.append(p1)
        return len(pts0) - 1

    for k, gap in enumerate([0.0, 1e-12, 1e-9, 1e-7]):
        o = np.array([3.0 * k, 0.0, 0.0])
        a0 = add(o + (0, 0, 0.5), o + (0, 0, -0.5 + gap))
        a1 = add(o + (1, 0, 0.5), o + (1, 0, -0.5 + gap))
        b0 = add(o + (0.25, 0, 0), o + (0.25, 0, 0))
        b1 = add(o + (1.25, 0, 0), o + (1.25, 0, 0))
        edges += [(a0, a1), (b0, b1)]
        # vertex sliding in the plane of a triangle
        o2 = o + (0, 5, 0)
        p = add(o2 + (-0.5, 0.2, gap), o2 + (1.5, 0.2, gap))
        t = [add(o2 + (0, 0, 0), o2 + (0, 0, 0)), add(o2 + (1, 0, 0), o2 + (1, 0, 0)), add(o2 + (0, 1, 0), o2 + (0, 1, 0))]
        faces.append(t)
        del p
    V0 = np.array(pts0, float)
    V1 = np.array(pts1, float)
    F = np.array(faces, np.int32)
    E = np.array(edges, np.int32)
    return scenes.Scene("degenerate", V0, V1, E, F)


@pytest.mark.parametrize("max_iter", [1, 10, 1000, 100000, 10 ** 6])
def test_narrow_degenerate_caps(ctx, max_iter):
    s = _degenerate_scene()
    vf, ee = oracle.all_pairs(s.E, s.F, s.nv)
    oh, ot, on_ = check_narrow(ctx, s, vf, ee, max_iter=max_iter)
    assert oh.any()


def test_narrow_order_independent(ctx):
    s = scenes.two_spheres()
    vf, ee = oracle.broad(s.V0, s.V1, s.E, s.F)
    h1, t1, m1, n1 = run_narrow(ctx, s, vf, ee)
    rng = np.random.default_rng(3)
    pv, pe = rng.permutation(len(vf)), rng.permutation(len(ee))
    h2, t2, m2, n2 = run_narrow(ctx, s, vf[pv], ee[pe])
    perm = np.concatenate([pv, len(vf) + pe])
    assert np.array_equal(h2, h1[perm]) and np.array_equal(t2.view(np.int64), t1[perm].view(np.int64))
    assert np.array_equal(n2, n1[perm]) and m1 == m2


def test_calls_on_two_streams_while_pools_grow():
    """A fresh context called alternately on two streams with growing scenes, so that each call grows
    scratch pools (freed and reallocated on its own stream) that the previous call on the other stream used:
    every result equals the same call's on the default stream (calls of one context run in call order)."""
    scs = [scenes.cloth_on_sphere(n=n, sphere_subdivisions=k, seed=50 + n) for n, k in ((9, 1), (33, 2), (65, 3),
                                                                                     (129, 3))]
    ref_ctx = ccd.Context(0)
    refs = []
    try:
        for s in scs:
            vf, ee = run_broad(ref_ctx, s)
            hit, toi, tmin, nenq = run_narrow(ref_ctx, s, vf, ee)
            refs.append((vf, ee, hit, toi.view(np.int64), tmin, nenq))
    finally:
        ref_ctx.close()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    c = ccd.Context(0)
    try:
        for i, (s, ref) in enumerate(zip(scs, refs)):
            st = streams[i % 2]
            vf, ee = run_broad(c, s, stream=st)
            assert np.array_equal(vf, ref[0]) and np.array_equal(ee, ref[1])
            hit, toi, tmin, nenq = c.narrow(dev(s.V0, torch.float64), dev(s.V1, torch.float64), dev(s.E, torch.int32),
                                            dev(s.F, torch.int32), dev(vf, torch.int32), dev(ee, torch.int32),
                                            DELTA, 10 ** 6, with_costs=True, stream=st)
            st.synchronize()
            assert np.array_equal(hit.cpu().numpy(), ref[2])
            assert np.array_equal(toi.cpu().numpy().view(np.int64), ref[3])
            assert float(tmin.cpu()[0]) == ref[4] or (np.isinf(ref[4]) and np.isinf(float(tmin.cpu()[0])))
            assert np.array_equal(nenq.cpu().numpy(), ref[5])
    finally:
        c.close()


def test_narrow_empty_and_errors(ctx):
    s = scenes.tiny_random_scene(2, n_tris=5)
    z = np.zeros((0, 2), np.int32)
    h, t, m, n = run_narrow(ctx, s, z, z)
    assert len(h) == 0 and m == np.inf
    with pytest.raises(ccd.CCDError) as ei:
        run_narrow(ctx, s, np.array([[0, s.nf]], np.int32), z)
    assert ei.value.status == ccd.CCD_ERR_INVALID_ARG
    with pytest.raises(ccd.CCDError) as ei:
        run_narrow(ctx, s, z, np.array([[0, 1]], np.int32), delta=0.0)
    assert ei.value.status == ccd.CCD_ERR_INVALID_ARG
    with pytest.raises(ccd.CCDError) as ei:
        run_narrow(ctx, s, z, np.array([[0, 1]], np.int32), max_iter=0)
    assert ei.value.status == ccd.CCD_ERR_INVALID_ARG


def test_end_to_end_cloth(ctx):
    """Broad then narrow on the GPU, compared with oracle broad then oracle narrow."""
    s = scenes.cloth_on_sphere(n=96, sphere_subdivisions=3, seed=21)
    V0, V1 = dev(s.V0, torch.float64), dev(s.V1, torch.float64)
    E, F = dev(s.E, torch.int32), dev(s.F, torch.int32)
    gvf, gee = ctx.broad(V0, V1, E, F)
    hit, toi, tmin, nenq = ctx.narrow(V0, V1, E, F, gvf, gee, DELTA, 10 ** 6, with_costs=True)
    ovf, oee = oracle.broad(s.V0, s.V1, s.E, s.F)
    oh, ot, on_, _, omin = oracle.narrow(s.V0, s.V1, s.E, s.F, ovf, oee)
    assert np.float64(tmin.cpu()[0]).view(np.int64) == np.float64(omin).view(np.int64)
    # per-pair results keyed by pair, vertex-face and edge-edge
    nvf = len(gvf)
    hit, toi, nenq = hit.cpu().numpy(), toi.cpu().numpy().view(np.int64), nenq.cpu().numpy()
    g = {("vf",) + tuple(p): (hit[i], toi[i], nenq[i]) for i, p in enumerate(gvf.cpu().numpy())}
    g.update({("ee",) + tuple(p): (hit[nvf + i], toi[nvf + i], nenq[nvf + i])
              for i, p in enumerate(gee.cpu().numpy())})
    assert len(g) == len(ovf) + len(oee)
    ot = ot.view(np.int64)
    for i, p in enumerate(ovf):
        assert g[("vf",) + tuple(p)] == (oh[i], ot[i], on_[i])
    for i, p in enumerate(oee):
        j = len(ovf) + i
        assert g[("ee",) + tuple(p)] == (oh[j], ot[j], on_[j])


@pytest.mark.parametrize("tuning", [{"heavy_lds": 1}, {"heavy_lds": 1, "heavy_cap_log2": 8, "heavy_slots": 16},
                                    {"sweep_tile_group": 1, "pool_blocks_per_cu": 1},
                                    {"heavy_block": 64, "heavy_slots": 4096, "heavy_lds": 1},
                                    {"heavy_block": 64, "heavy_cap_log2": 8, "pool_wait": 1},
                                    {"heavy_lds": 0, "pool_wait": 1, "heavy_cap_log2": 17},
                                    {"heavy_block": 1024, "heavy_slots": 256},
                                    {"heavy_block": 1024, "heavy_lds": 0, "heavy_cap_log2": 10},
                                    {"heavy_block": 256},
                                    {"pool_wait": 0}, {"pool_wait": 4, "heavy_cap_log2": 8},
                                    {"pool_root_limit": 16}, {"pool_root_limit": 320, "pool_wait": 0}])
def test_tunings_give_identical_results(ctx, tuning):
    """Launch shapes (LDS frontiers, tiny wide-stage buffers that force re-runs, one pool workgroup per CU,
    ungrouped sweep tiles, one-wave wide-stage workgroups, pool pairs that never wait, always wait or wait
    only when they have few children, pool root admission limits from 16 to 320) never change a result."""
    print(f"tuning {tuning}", flush=True)
    ctx.set_tuning(tuning)
    try:
        s = _degenerate_scene()
        vf, ee = oracle.all_pairs(s.E, s.F, s.nv)
        for max_iter in (1000, 10 ** 6):
            oh, _, _ = check_narrow(ctx, s, vf, ee, max_iter=max_iter)
            assert oh.any()
        s = scenes.cloth_on_sphere(n=96, sphere_subdivisions=3, seed=21)
        ovf, oee = check_broad(ctx, s)
        check_narrow(ctx, s, ovf, oee)
    finally:
        ctx.set_tuning(None)


@pytest.mark.parametrize("tuning", [None, {"heavy_lds": 0}, {"heavy_block": 64}, {"heavy_block": 1024},
                                    {"heavy_cap_log2": 8, "heavy_slots": 16}])
def test_narrow_levels_past_21(ctx, tuning):
    """Pairs whose split levels m_k are at most 21 but whose search splits past level 21 (coordinates near
    2^33 keep the inclusion box wider than delta): the wide stage must switch its frontier layout when a
    level first exceeds 21.  Every pair compared with the oracle bit for bit."""
    from test_oracle_pins import DEEP_SEEDS
    if tuning:
        ctx.set_tuning(tuning)
    try:
        for delta in (1.07e-6, 1e-6):
            vq = [deep_split_query(sd, 0)[0] for sd in DEEP_SEEDS[0][delta]]
            eq = [deep_split_query(sd, 1)[0] for sd in DEEP_SEEDS[1][delta]]
            V0, V1, E, F, vf, ee = scene_of_queries(vq, eq)
            s = scenes.Scene("deep_levels", V0, V1, E, F)
            oh, _, _ = check_narrow(ctx, s, vf, ee, delta=delta)
            assert oh.all()
            assert ctx.stats()["heavy_pairs"] == len(vf) + len(ee)  # every pair went past the pool's 21 levels
    finally:
        ctx.set_tuning(None)
