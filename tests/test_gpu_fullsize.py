"""The full-size workloads on the GPU, checked against the oracle where it can follow.

The 1M-triangle perturbed torus (with near-degenerate gadgets inside the tube)
and the 64-scene batch are too large for the oracle's brute-force broad phase
and for its narrow phase on every pair, so:
  * broad phase: for sampled vertices, faces and edges, every overlapping
    partner found by brute force over all boxes (the oracle's boxes) must be
    among the GPU's pairs and vice versa;
  * narrow phase: on a uniform sample of the GPU's pairs plus a sample of the
    gadget pairs, hit / toi / n_enq must equal the oracle's bit for bit, and the
    reported minimum must be the minimum of the per-pair times.
"""
import numpy as np
import pytest

import oracle
import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2112_06300_amd as ccd  # noqa: E402

DELTA = 1e-6
GADGETS = 9000


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ccd.Context(0)
    yield c
    c.close()


def dev(x, dt):
    return torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dt)


def pair_set(a):
    a = np.asarray(a, np.int64).reshape(-1, 2)
    return set(map(tuple, a.tolist()))


def check_broad_sampled(s, vf, ee, rng, n_sample=200):
    lo, hi = oracle.boxes(s.V0, s.V1, s.E, s.F)
    nv, ne = s.nv, s.ne
    lv, hv = lo[:nv], hi[:nv]
    le, he = lo[nv:nv + ne], hi[nv:nv + ne]
    lf, hf = lo[nv + ne:], hi[nv + ne:]
    F = np.asarray(s.F, np.int64)
    E = np.asarray(s.E, np.int64)
    by_v, by_f, by_e = {}, {}, {}
    for v, f in vf:
        by_v.setdefault(v, set()).add(f)
        by_f.setdefault(f, set()).add(v)
    for e, g in ee:
        by_e.setdefault(e, set()).add(g)
        by_e.setdefault(g, set()).add(e)
    for v in rng.choice(nv, n_sample, replace=False):
        hit = np.nonzero(np.all((lf <= hv[v]) & (lv[v] <= hf), axis=1))[0]
        hit = hit[~np.any(F[hit] == v, axis=1)]
        assert set(hit.tolist()) == by_v.get(v, set()), ("vertex", v)
    for f in rng.choice(s.nf, n_sample, replace=False):
        hit = np.nonzero(np.all((lv <= hf[f]) & (lf[f] <= hv), axis=1))[0]
        hit = hit[~np.isin(hit, F[f])]
        assert set(hit.tolist()) == by_f.get(f, set()), ("face", f)
    for e in rng.choice(ne, n_sample, replace=False):
        hit = np.nonzero(np.all((le <= he[e]) & (le[e] <= he), axis=1))[0]
        share = (E[hit, 0] == E[e, 0]) | (E[hit, 0] == E[e, 1]) | (E[hit, 1] == E[e, 0]) | (E[hit, 1] == E[e, 1])
        hit = hit[~share & (hit != e)]
        assert set(hit.tolist()) == by_e.get(e, set()), ("edge", e)


def check_narrow_sampled(s, vf, ee, hit, toi, nenq, idx):
    nvf = len(vf)
    svf = vf[idx[idx < nvf]]
    see = ee[idx[idx >= nvf] - nvf]
    oh, ot, on_, _, _ = oracle.narrow(s.V0, s.V1, s.E, s.F, svf, see, DELTA)
    order = np.concatenate([idx[idx < nvf], idx[idx >= nvf]])
    assert np.array_equal(hit[order], oh)
    assert np.array_equal(toi[order].view(np.int64), ot.view(np.int64))
    assert np.array_equal(nenq[order], on_)


def test_torus_with_gadgets_sampled(ctx):
    s = scenes.perturbed_torus(gadgets=GADGETS)
    print(f"torus: nv={s.nv} ne={s.ne} nf={s.nf} gadgets={GADGETS}", flush=True)
    V0, V1, E, F = dev(s.V0, torch.float64), dev(s.V1, torch.float64), dev(s.E, torch.int32), dev(s.F, torch.int32)
    gvf, gee = ctx.broad(V0, V1, E, F, vf_cap=60_000_000, ee_cap=200_000_000)
    hit, toi, tmin, nenq = ctx.narrow(V0, V1, E, F, gvf, gee, DELTA, 10 ** 6, with_costs=True)
    torch.cuda.synchronize()
    vf, ee = gvf.cpu().numpy(), gee.cpu().numpy()
    hit, toi, nenq = hit.cpu().numpy(), toi.cpu().numpy(), nenq.cpu().numpy()
    tmin = float(tmin.cpu()[0])
    print(f"pairs {len(vf)} + {len(ee)}, hits {int(hit.sum())}, capped {int((nenq > 10 ** 6).sum())}", flush=True)
    # no pair is reported twice
    assert len(pair_set(vf)) == len(vf) and len(pair_set(ee)) == len(ee)
    rng = np.random.Generator(np.random.PCG64(31))
    check_broad_sampled(s, vf, ee, rng)
    # narrow: uniform sample plus gadget pairs (vertex ids past the torus)
    torus_nv = 1000 * 500
    n = len(vf) + len(ee)
    gad = np.concatenate([np.nonzero(vf[:, 0] >= torus_nv)[0], len(vf) + np.nonzero(
        np.asarray(s.E)[ee[:, 0], 0] >= torus_nv)[0]])
    assert len(gad) > 0
    idx = np.unique(np.concatenate([rng.choice(n, 3000, replace=False), rng.choice(gad, min(120, len(gad)),
                                                                                   replace=False)]))
    check_narrow_sampled(s, vf, ee, hit, toi, nenq, idx)
    assert np.float64(tmin).view(np.int64) == np.float64(toi.min()).view(np.int64)
    # the gadgets are near-degenerate by construction: some of their pairs hit the cap
    assert (nenq[gad] > 10 ** 6).any()


def test_scene_batch_64_sampled(ctx):
    scs = scenes.scene_batch()
    V0, V1, E, F, vo, eo, fo = scenes.concat_scenes(scs)
    nb = int(vo[-1] + eo[-1] + fo[-1])
    print(f"batch: {len(scs)} scenes, {int(fo[-1])} triangles, {nb} boxes", flush=True)
    b = ccd.Batch(ctx, vo, eo, fo, 3 * nb, 6 * nb)
    inp = (dev(V0, torch.float64), dev(V1, torch.float64), dev(E, torch.int32), dev(F, torch.int32))
    vf, ee, hit, toi, tmin, nenq = b.run(*inp, DELTA, 10 ** 6, use_graph=True, with_costs=True)
    torch.cuda.synchronize()
    vf, ee = vf.cpu().numpy(), ee.cpu().numpy()
    hit, toi, tmin, nenq = hit.cpu().numpy(), toi.cpu().numpy(), tmin.cpu().numpy(), nenq.cpu().numpy()
    rng = np.random.Generator(np.random.PCG64(41))
    nvf = len(vf)
    sv = np.searchsorted(vo, vf[:, 0], side="right") - 1
    se = np.searchsorted(eo, ee[:, 0], side="right") - 1
    for i in rng.choice(len(scs), 8, replace=False):
        s = scs[i]
        print(f"scene {i}: {s.name} nf={s.nf}", flush=True)
        mv, me = np.nonzero(sv == i)[0], np.nonzero(se == i)[0]
        lvf = vf[mv] - np.array([vo[i], fo[i]])
        lee = ee[me] - eo[i]
        check_broad_sampled(s, lvf, lee, rng, n_sample=100)
        # narrow on a sample of the scene's pairs, in the scene's own ids
        k = min(400, len(mv) + len(me))
        pick = rng.choice(len(mv) + len(me), k, replace=False)
        gidx = np.concatenate([mv, nvf + me])[pick]
        loc = np.concatenate([np.arange(len(mv)), len(mv) + np.arange(len(me))])[pick]
        svf = lvf[loc[loc < len(mv)]]
        see = lee[loc[loc >= len(mv)] - len(mv)]
        oh, ot, on_, _, _ = oracle.narrow(s.V0, s.V1, s.E, s.F, svf, see, DELTA)
        order = np.concatenate([gidx[loc < len(mv)], gidx[loc >= len(mv)]])
        assert np.array_equal(hit[order], oh)
        assert np.array_equal(toi[order].view(np.int64), ot.view(np.int64))
        assert np.array_equal(nenq[order], on_)
        # the scene's minimum is the minimum over its pairs
        own = np.concatenate([toi[mv], toi[nvf + me]])
        ref = own.min() if len(own) else np.inf
        assert np.float64(tmin[i]).view(np.int64) == np.float64(ref).view(np.int64)
    b.close()


def test_learned_schedule_10M_pairs_identical(ctx):
    """10M candidate pairs drawn from the perturbed torus's candidates (degenerate share kept): the learned
    schedule's outputs equal the plain schedule's on every pair, and the oracle's on a sample."""
    from paper_2112_06300_amd import sched
    s = scenes.perturbed_torus(seed=5, gadgets=sched.TORUS_GADGETS)
    V0, V1, E, F = dev(s.V0, torch.float64), dev(s.V1, torch.float64), dev(s.E, torch.int32), dev(s.F, torch.int32)
    cvf, cee = ctx.broad(V0, V1, E, F, vf_cap=60_000_000, ee_cap=200_000_000)
    vf, ee = scenes.sample_pairs(cvf.cpu().numpy(), cee.cpu().numpy(), 10_000_000, seed=5)
    print(f"10M pairs: {len(vf)} VF + {len(ee)} EE", flush=True)
    try:
        params, norm, _ = sched.load_model(sched.TORUS_MODEL_PATH)
    except FileNotFoundError:
        params, norm, _ = sched.load_model()
    dvf, dee = dev(vf, torch.int32), dev(ee, torch.int32)
    plain = [x.cpu().numpy() for x in ctx.narrow(V0, V1, E, F, dvf, dee, DELTA, 10 ** 6, with_costs=True)]
    learned = [x.cpu().numpy() for x in ctx.narrow(V0, V1, E, F, dvf, dee, DELTA, 10 ** 6, with_costs=True,
                                                  schedule=("learned", params, norm))]
    st = ctx.stats()
    print(f"learned: {st['sched_heavy_pairs']} pairs started in the wide stage", flush=True)
    assert np.array_equal(plain[0], learned[0])
    assert np.array_equal(plain[1].view(np.int64), learned[1].view(np.int64))
    assert np.array_equal(plain[2].view(np.int64), learned[2].view(np.int64))
    assert np.array_equal(plain[3], learned[3])
    rng = np.random.Generator(np.random.PCG64(51))
    idx = np.unique(rng.choice(len(vf) + len(ee), 2000, replace=False))
    check_narrow_sampled(s, vf, ee, plain[0], plain[1], plain[3], idx)


def test_detect_bench_workload_matches_oracle(ctx):
    """The timed step of the benchmark -- ccd_detect with the learned schedule on the 256 x 256 cloth and
    the 10,242-vertex sphere, with the capacities and launch shapes the benchmark uses -- against the
    oracle's brute-force broad phase and narrow phase on every pair: identical pair sets, per-pair
    hit / toi / n_enq bit for bit, and the minimum."""
    from paper_2112_06300_amd import sched
    s = scenes.cloth_on_sphere()
    print(f"detect full size: {s.name} nv={s.nv} ne={s.ne} nf={s.nf}", flush=True)
    V0, V1, E, F = dev(s.V0, torch.float64), dev(s.V1, torch.float64), dev(s.E, torch.int32), dev(s.F, torch.int32)
    ovf, oee = oracle.broad(s.V0, s.V1, s.E, s.F)
    cap_vf, cap_ee = len(ovf) + 1024, len(oee) + 1024
    vf = torch.empty((cap_vf, 2), dtype=torch.int32, device="cuda")
    ee = torch.empty((cap_ee, 2), dtype=torch.int32, device="cuda")
    n = cap_vf + cap_ee
    hit = torch.empty(n, dtype=torch.uint8, device="cuda")
    toi = torch.empty(n, dtype=torch.float64, device="cuda")
    tmin = torch.empty(1, dtype=torch.float64, device="cuda")
    nenq = torch.empty(n, dtype=torch.int64, device="cuda")
    p, nm, _ = sched.load_model()
    sc = ccd.prepare_schedule(("learned", dev(p, torch.float32), dev(nm, torch.float32), ccd.HEAVY_THRESHOLD,
                               ccd.MAX_HEAVY))
    n_vf, n_ee = ctx.detect_into(V0, V1, E, F, vf, ee, hit, toi, tmin, nenq, DELTA, 10 ** 6, schedule=sc)
    torch.cuda.synchronize()
    assert (n_vf, n_ee) == (len(ovf), len(oee))
    gvf, gee = vf[:n_vf].cpu().numpy(), ee[:n_ee].cpu().numpy()
    assert pair_set(gvf) == pair_set(ovf) and pair_set(gee) == pair_set(oee)
    oh, ot, on_, _, omin = oracle.narrow(s.V0, s.V1, s.E, s.F, gvf, gee, DELTA)
    m = n_vf + n_ee
    h, t, e = hit[:m].cpu().numpy(), toi[:m].cpu().numpy(), nenq[:m].cpu().numpy()
    assert np.array_equal(h, oh), np.nonzero(h != oh)[0][:10]
    assert np.array_equal(t.view(np.int64), ot.view(np.int64)), np.nonzero(t != ot)[0][:10]
    assert np.array_equal(e, on_), np.nonzero(e != on_)[0][:10]
    assert np.float64(tmin.cpu()[0]).view(np.int64) == np.float64(omin).view(np.int64)


def _torus_manifest(s):
    """The oracle's answer on the 1M-triangle torus with 12,000 gadgets: the committed manifest when its input
    hash matches these inputs, else computed now by the same oracle-only script (slow: tens of minutes)."""
    import json
    import os
    import sys
    here = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
    sys.path.insert(0, here)
    import make_torus_manifest as mk
    try:
        man = json.load(open(mk.OUT))
    except (OSError, ValueError):
        man = None
    if man is None or man.get("input_sha256") != mk.scene_hash(s):
        print("manifest missing or stale: running the oracle on the full workload", flush=True)
        vf, ee = oracle.broad(s.V0, s.V1, s.E, s.F)
        hit, toi, n_enq, _, _, tmin = oracle.narrow_with_work(s.V0, s.V1, s.E, s.F, vf, ee, DELTA, 10 ** 6)
        capped = n_enq > 10 ** 6
        man = {"n_vf": len(vf), "n_ee": len(ee), "pairs_sha256": mk.pairs_hash(vf, ee),
               "results_sha256": mk.results_hash(vf, ee, hit, toi, n_enq),
               "toi_min_bits": int(np.float64(tmin).view(np.int64)), "capped_pairs": int(capped.sum()),
               "toi_min_from_capped_pair": bool(np.any(capped & (toi == tmin))),
               "toi_min_uncapped": float(toi[~capped].min()) if np.any(~capped) else float("inf")}
    return mk, man


@pytest.mark.timeout(1800)
def test_torus_with_gadgets_full(ctx):
    """The benchmark's workload whole: ccd_detect (learned schedule, as timed, and plain) on the 1M-triangle torus
    with 12,000 near-degenerate gadgets.  The candidate set and every pair's hit, TOI bits and n_enq equal the
    oracle's (brute-force broad phase, per-pair narrow phase), compared through hashes of the canonically
    sorted pairs and results; the earliest time is identical; Alg. 3's single shared t* gives the same earliest
    time when the oracle's earliest pair is not a capped one, and stays within the allowed range otherwise."""
    from paper_2112_06300_amd import sched
    s = scenes.perturbed_torus(seed=3, gadgets=sched.TORUS_GADGETS)
    print(f"torus full: nv={s.nv} ne={s.ne} nf={s.nf}", flush=True)
    mk, man = _torus_manifest(s)
    V0, V1, E, F = dev(s.V0, torch.float64), dev(s.V1, torch.float64), dev(s.E, torch.int32), dev(s.F, torch.int32)
    cap_vf, cap_ee = man["n_vf"] + 1024, man["n_ee"] + 1024
    vf = torch.empty((cap_vf, 2), dtype=torch.int32, device="cuda")
    ee = torch.empty((cap_ee, 2), dtype=torch.int32, device="cuda")
    n = cap_vf + cap_ee
    hit = torch.empty(n, dtype=torch.uint8, device="cuda")
    toi = torch.empty(n, dtype=torch.float64, device="cuda")
    tmin = torch.empty(1, dtype=torch.float64, device="cuda")
    nenq = torch.empty(n, dtype=torch.int64, device="cuda")
    p, nm, _ = sched.load_model(sched.TORUS_MODEL_PATH)
    learned = ccd.prepare_schedule(("learned", dev(p, torch.float32), dev(nm, torch.float32),
                                    ccd.TORUS_HEAVY_THRESHOLD, ccd.TORUS_MAX_HEAVY))
    for name, sc in (("learned", learned), ("plain", None)):
        n_vf, n_ee = ctx.detect_into(V0, V1, E, F, vf, ee, hit, toi, tmin, nenq, DELTA, 10 ** 6, schedule=sc)
        torch.cuda.synchronize()
        print(f"{name}: {n_vf} + {n_ee} pairs, stats {ctx.stats()}", flush=True)
        assert (n_vf, n_ee) == (man["n_vf"], man["n_ee"])
        gvf, gee = vf[:n_vf].cpu().numpy(), ee[:n_ee].cpu().numpy()
        m = n_vf + n_ee
        assert mk.pairs_hash(gvf, gee) == man["pairs_sha256"]
        assert mk.results_hash(gvf, gee, hit[:m].cpu().numpy(), toi[:m].cpu().numpy(),
                               nenq[:m].cpu().numpy()) == man["results_sha256"]
        assert int(np.float64(tmin.cpu()[0]).view(np.int64)) == man["toi_min_bits"]
    # Alg. 3's shared t*
    ctx.detect_into(V0, V1, E, F, vf, ee, hit, toi, tmin, None, DELTA, 10 ** 6, options={"earliest_only": 1})
    g = float(tmin.cpu()[0])
    o = float(np.int64(man["toi_min_bits"]).view(np.float64))
    if not man["toi_min_from_capped_pair"]:
        assert np.float64(g).view(np.int64) == man["toi_min_bits"]
    else:
        assert o <= g <= man["toi_min_uncapped"]
