"""Batches of scenes (CSR layout, one pass, optionally a captured graph) through the C ABI.

Every scene of a batch must give exactly what it gives alone: the same
candidate pairs (in its own ids), the same per-pair hit / toi / n_enq and the
same earliest time of impact; small batches are also checked against the
oracle scene by scene.
"""
import os

import numpy as np
import pytest

import oracle
import scenes

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


def dev(x, dt):
    return torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dt)


def small_batch(seed=4, count=6, t_min=200, t_max=6000):
    return scenes.scene_batch(seed=seed, count=count, t_min=t_min, t_max=t_max)


def batch_inputs(scs):
    V0, V1, E, F, vo, eo, fo = scenes.concat_scenes(scs)
    return (dev(V0, torch.float64), dev(V1, torch.float64), dev(E, torch.int32), dev(F, torch.int32)), (vo, eo, fo)


def split_results(vf, ee, hit, toi, nenq, offs, S):
    """Per scene: dict (kind, a, b) in local ids -> (hit, toi bits, n_enq)."""
    vo, eo, fo = offs
    vf, ee = vf.cpu().numpy(), ee.cpu().numpy()
    hit, toi = hit.cpu().numpy(), toi.cpu().numpy().view(np.int64)
    nenq = nenq.cpu().numpy()
    out = [dict() for _ in range(S)]
    nvf = len(vf)
    for p, (v, f) in enumerate(vf):
        s = int(np.searchsorted(vo, v, side="right") - 1)
        assert fo[s] <= f < fo[s + 1], "pair crosses scenes"
        out[s][(0, v - vo[s], f - fo[s])] = (hit[p], toi[p], nenq[p])
    for q, (e, g) in enumerate(ee):
        s = int(np.searchsorted(eo, e, side="right") - 1)
        assert eo[s] <= g < eo[s + 1], "pair crosses scenes"
        out[s][(1, e - eo[s], g - eo[s])] = (hit[nvf + q], toi[nvf + q], nenq[nvf + q])
    return out


def single_results(ctx, s):
    V0, V1, E, F = dev(s.V0, torch.float64), dev(s.V1, torch.float64), dev(s.E, torch.int32), dev(s.F, torch.int32)
    vf, ee = ctx.broad(V0, V1, E, F)
    hit, toi, tmin, nenq = ctx.narrow(V0, V1, E, F, vf, ee, DELTA, 10 ** 6, with_costs=True)
    torch.cuda.synchronize()
    d = {}
    vf, ee = vf.cpu().numpy(), ee.cpu().numpy()
    h, t, n = hit.cpu().numpy(), toi.cpu().numpy().view(np.int64), nenq.cpu().numpy()
    for p, (v, f) in enumerate(vf):
        d[(0, v, f)] = (h[p], t[p], n[p])
    for q, (e, g) in enumerate(ee):
        d[(1, e, g)] = (h[len(vf) + q], t[len(vf) + q], n[len(vf) + q])
    return d, float(tmin.cpu()[0])


def make_batch(ctx, scs, offs, slack=2.0):
    vo, eo, fo = offs
    nb = int(vo[-1] + eo[-1] + fo[-1])
    cap = int(slack * 4 * nb) + 1024
    return ccd.Batch(ctx, vo, eo, fo, cap, cap)


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_equals_scenes_alone(ctx, use_graph):
    scs = small_batch()
    inp, offs = batch_inputs(scs)
    print(f"batch: {len(scs)} scenes, faces {[s.nf for s in scs]}, graph={use_graph}", flush=True)
    b = make_batch(ctx, scs, offs)
    vf, ee, hit, toi, tmin, nenq = b.run(*inp, DELTA, 10 ** 6, use_graph=use_graph, with_costs=True)
    torch.cuda.synchronize()
    per = split_results(vf, ee, hit, toi, nenq, offs, len(scs))
    tmin = tmin.cpu().numpy()
    for i, s in enumerate(scs):
        alone, amin = single_results(ctx, s)
        assert per[i].keys() == alone.keys(), (i, len(per[i]), len(alone))
        for k, v in alone.items():
            assert per[i][k] == v, (i, k, per[i][k], v)
        assert np.float64(tmin[i]).view(np.int64) == np.float64(amin).view(np.int64), (i, tmin[i], amin)
    b.close()


def test_batch_matches_oracle(ctx):
    scs = [scenes.tiny_random_scene(s, n_tris=10, extent=0.5, motion=1.0) for s in (21, 22, 23)]
    scs.append(scenes.two_spheres(subdivisions=1))
    inp, offs = batch_inputs(scs)
    b = make_batch(ctx, scs, offs)
    vf, ee, hit, toi, tmin, nenq = b.run(*inp, DELTA, 10 ** 6, with_costs=True)
    per = split_results(vf, ee, hit, toi, nenq, offs, len(scs))
    tmin = tmin.cpu().numpy()
    for i, s in enumerate(scs):
        ovf, oee = oracle.broad(s.V0, s.V1, s.E, s.F)
        oh, ot, on_, _, omin = oracle.narrow(s.V0, s.V1, s.E, s.F, ovf, oee, DELTA)
        ref = {(0, v, f): (oh[p], ot[p:p + 1].view(np.int64)[0], on_[p]) for p, (v, f) in enumerate(ovf)}
        ref.update({(1, e, g): (oh[len(ovf) + q], ot[len(ovf) + q:len(ovf) + q + 1].view(np.int64)[0],
                                on_[len(ovf) + q]) for q, (e, g) in enumerate(oee)})
        assert per[i] == ref, i
        assert np.float64(tmin[i]).view(np.int64) == np.float64(omin).view(np.int64)


def canonical(b, res, offs):
    """Per-scene results keyed by pair (the sweep emits pairs in any order) and toi_min bits."""
    vf, ee, hit, toi, tmin, nenq = res
    if nenq is None:
        nenq = torch.zeros(hit.shape[0], dtype=torch.int64, device=hit.device)
    per = split_results(vf, ee, hit, toi, nenq, offs, b.n_scenes)
    return per, tmin.cpu().numpy().view(np.int64).tolist()


def test_graph_replays_match_eager(ctx):
    scs = small_batch(seed=5, count=5)
    inp, offs = batch_inputs(scs)
    b = make_batch(ctx, scs, offs)
    ref = canonical(b, b.run(*inp, DELTA, 10 ** 6, use_graph=False, with_costs=True), offs)
    assert sum(len(d) for d in ref[0]) > 0
    for it in range(4):
        # the program's own eager work between replays
        junk = torch.randn(1 << 20, device="cuda").sum()
        torch.cuda.synchronize()
        got = canonical(b, b.run(*inp, DELTA, 10 ** 6, use_graph=True, with_costs=True), offs)
        assert got == ref, it
        del junk
    # a tuning change re-captures; results do not change
    ctx.set_tuning({"sweep_tile_group": 4, "heavy_slots": 256})
    try:
        assert canonical(b, b.run(*inp, DELTA, 10 ** 6, use_graph=True, with_costs=True), offs) == ref
    finally:
        ctx.set_tuning(None)
    b.close()


def test_single_scene_batch_and_empty_scenes(ctx):
    s = scenes.cloth_on_sphere(seed=7, n=24, sphere_subdivisions=2)
    empty = scenes.Scene("empty", np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 2), np.int32),
                         np.zeros((0, 3), np.int32))
    far = scenes.tiny_random_scene(3, n_tris=1)   # one triangle: no pairs at all
    for scs in ([s], [empty, s, empty], [far, empty]):
        inp, offs = batch_inputs(scs)
        b = make_batch(ctx, scs, offs)
        vf, ee, hit, toi, tmin, nenq = b.run(*inp, DELTA, 10 ** 6, with_costs=True)
        per = split_results(vf, ee, hit, toi, nenq, offs, len(scs))
        tmin = tmin.cpu().numpy()
        for i, sc in enumerate(scs):
            if sc.nf == 0 or sc.name == "tiny_random":
                assert per[i] == {} and np.isinf(tmin[i])
            else:
                alone, amin = single_results(ctx, sc)
                assert per[i] == alone
                assert tmin[i] == amin
        b.close()


def test_capacity_error_reports_required_counts(ctx):
    scs = small_batch(seed=6, count=3)
    inp, offs = batch_inputs(scs)
    vo, eo, fo = offs
    b = ccd.Batch(ctx, vo, eo, fo, 16, 16)
    with pytest.raises(ccd.CCDError) as e:
        b.run(*inp, DELTA, 10 ** 6)
    assert e.value.status == ccd.CCD_ERR_CAPACITY
    need_vf, need_ee = b.n_vf, b.n_ee
    assert need_vf > 16 or need_ee > 16
    b.close()
    b = ccd.Batch(ctx, vo, eo, fo, need_vf, need_ee)
    vf, ee, *_ = b.run(*inp, DELTA, 10 ** 6)
    assert len(vf) == need_vf and len(ee) == need_ee
    b.close()


def test_face_using_another_scenes_vertex_is_rejected(ctx):
    scs = [scenes.tiny_random_scene(s, n_tris=3) for s in (1, 2)]
    V0, V1, E, F, vo, eo, fo = scenes.concat_scenes(scs)
    F = F.copy()
    F[0, 0] = vo[1]  # a vertex of scene 1 in a face of scene 0
    b = ccd.Batch(ctx, vo, eo, fo, 1024, 1024)
    with pytest.raises(ccd.CCDError) as e:
        b.run(dev(V0, torch.float64), dev(V1, torch.float64), dev(E, torch.int32), dev(F, torch.int32))
    assert e.value.status == ccd.CCD_ERR_INVALID_ARG
    b.close()


def test_autotune_sets_tuning_and_uses_cache(ctx, tmp_path):
    scs = small_batch(seed=7, count=4)
    inp, offs = batch_inputs(scs)
    b = make_batch(ctx, scs, offs)
    ref = canonical(b, b.run(*inp, DELTA, 10 ** 6, use_graph=False), offs)
    cache = str(tmp_path / "tune.txt")
    try:
        t = b.autotune(*inp, DELTA, 10 ** 6, cache_path=cache)
        assert t == ctx.get_tuning()
        lines = open(cache).read().splitlines()
        assert len(lines) == 1 and lines[0].startswith("gfx")
        ctx.set_tuning(None)
        t2 = b.autotune(*inp, DELTA, 10 ** 6, cache_path=cache)
        assert t2 == t and open(cache).read().splitlines() == lines  # taken from the cache
        assert canonical(b, b.run(*inp, DELTA, 10 ** 6, use_graph=True), offs) == ref
    finally:
        ctx.set_tuning(None)
    b.close()
