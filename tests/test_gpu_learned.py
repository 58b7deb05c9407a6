"""The learned schedule on the GPU, through the C ABI.

Features, the bf16 network's predictions, its gradients and the Adam step are
checked against the float64 CPU reference; every schedule (plain, learned,
caller-given order) must give bit-identical narrow-phase outputs, since a
permutation of the pairs cannot change any pair's canonical result.
"""
import numpy as np
import pytest

import oracle
import scenes
from oracle import sched_ref as R

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2112_06300_amd as ccd  # noqa: E402
from paper_2112_06300_amd import sched  # noqa: E402

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


def scene_dev(s):
    return dev(s.V0, torch.float64), dev(s.V1, torch.float64), dev(s.E, torch.int32), dev(s.F, torch.int32)


def random_model(seed, scale=0.3):
    rng = np.random.Generator(np.random.PCG64(seed))
    params = rng.normal(0.0, scale, R.N_PARAMS).astype(np.float32)
    norm = np.concatenate([rng.normal(0.0, 0.5, R.NF), rng.uniform(0.5, 1.5, R.NF)]).astype(np.float32)
    return params, norm


# --------------------------------------------------------------------------- features
@pytest.mark.parametrize("name", ["cloth", "spheres", "tiny"])
def test_features_match_reference(ctx, name):
    s = {"cloth": lambda: scenes.cloth_on_sphere(seed=7, n=16, sphere_subdivisions=2),
         "spheres": lambda: scenes.two_spheres(subdivisions=1),
         "tiny": lambda: scenes.tiny_random_scene(5, n_tris=8, extent=0.5, motion=1.0)}[name]()
    vf, ee = oracle.broad(s.V0, s.V1, s.E, s.F)
    print(f"features: {name} pairs={len(vf)}+{len(ee)}", flush=True)
    assert len(vf) + len(ee) > 0
    g = ctx.features(*scene_dev(s), dev(vf, torch.int32), dev(ee, torch.int32), DELTA).cpu().numpy()
    ref = R.pair_features(s.V0, s.V1, s.E, s.F, vf, ee, DELTA)
    # discrete features come from the same canonical float64 evaluation: identical
    for k in (0, 1, 2, 3, 10, 14):
        assert np.array_equal(g[:, k], ref[:, k]), (k, np.nonzero(g[:, k] != ref[:, k])[0][:5])
    # logarithms and the cosine: float64 values rounded to float32 on both sides
    np.testing.assert_allclose(g, ref, rtol=2e-6, atol=2e-6)


def test_features_reject_bad_pair(ctx):
    s = scenes.tiny_random_scene(5, n_tris=4)
    vf = np.array([[0, 1], [0, 99]], np.int32)
    with pytest.raises(ccd.CCDError) as e:
        ctx.features(*scene_dev(s), dev(vf, torch.int32), torch.zeros((0, 2), dtype=torch.int32, device="cuda"))
    assert e.value.status == ccd.CCD_ERR_INVALID_ARG


# --------------------------------------------------------------------------- network
@pytest.mark.parametrize("n", [1, 16, 1013, 40000])
def test_predict_matches_reference(ctx, n):
    params, norm = random_model(1)
    rng = np.random.Generator(np.random.PCG64(2))
    feat = rng.normal(0.0, 2.0, (n, R.NF)).astype(np.float32)
    print(f"predict: n={n}", flush=True)
    y = ctx.mlp_predict(dev(params, torch.float32), dev(norm, torch.float32), dev(feat, torch.float32))
    y = y.cpu().numpy().astype(np.float64)
    x = R.normalize(feat, norm)
    q = R.quantized(params)
    ref_rounded = R.forward(q, x, round_h1=True)   # the network exactly as evaluated, in float64
    ref_smooth = R.forward(q, x)
    scale = 1.0 + np.abs(ref_rounded)
    err = np.abs(y - ref_rounded) / scale
    # float32 accumulation; a bf16 rounding of h1 can flip where z1 sits on a rounding boundary
    assert np.median(err) <= 1e-5 and err.max() <= 2e-2, (np.median(err), err.max())
    assert np.abs(y - ref_smooth).max() <= 5e-2 * scale.max()


def test_predict_empty(ctx):
    params, norm = random_model(1)
    out = ctx.mlp_predict(dev(params, torch.float32), dev(norm, torch.float32),
                          torch.zeros((0, R.NF), dtype=torch.float32, device="cuda"))
    assert out.numel() == 0


@pytest.mark.parametrize("n", [7, 2005, 70001])
def test_gradient_matches_reference(ctx, n):
    params, norm = random_model(3)
    rng = np.random.Generator(np.random.PCG64(4))
    feat = rng.normal(0.0, 2.0, (n, R.NF)).astype(np.float32)
    label = rng.normal(2.0, 1.0, n).astype(np.float32)
    print(f"grad: n={n}", flush=True)
    g, sse = ctx.mlp_grad(dev(params, torch.float32), dev(norm, torch.float32), dev(feat, torch.float32),
                          dev(label, torch.float32))
    g = g.cpu().numpy().astype(np.float64)
    x = R.normalize(feat, norm)
    q = R.quantized(params)
    ref = R.grad(q, x, label.astype(np.float64))
    gp, rp = R.unpack(g), R.unpack(ref)
    for k, _ in R.SIZES:
        rel = np.linalg.norm(gp[k] - rp[k]) / max(np.linalg.norm(rp[k]), 1e-30)
        assert rel <= 1e-2, (k, rel)
    e = R.forward(q, x, round_h1=True) - label
    assert abs(float(sse.cpu()[0]) - float(e @ e)) <= 1e-3 * float(e @ e)


def test_gradient_of_no_rows_is_zero(ctx):
    params, norm = random_model(3)
    g, sse = ctx.mlp_grad(dev(params, torch.float32), dev(norm, torch.float32),
                          torch.zeros((0, R.NF), dtype=torch.float32, device="cuda"),
                          torch.zeros(0, dtype=torch.float32, device="cuda"))
    assert torch.count_nonzero(g).item() == 0 and float(sse.cpu()[0]) == 0.0


def test_adam_matches_reference(ctx):
    rng = np.random.Generator(np.random.PCG64(5))
    p0 = rng.normal(0, 0.3, R.N_PARAMS).astype(np.float32)
    grads = [rng.normal(0, 1, R.N_PARAMS).astype(np.float32) for _ in range(4)]
    p, m, v = dev(p0, torch.float32), torch.zeros(R.N_PARAMS, device="cuda"), torch.zeros(R.N_PARAMS, device="cuda")
    rp, rm, rv = p0.astype(np.float64), np.zeros(R.N_PARAMS), np.zeros(R.N_PARAMS)
    for step, gr in enumerate(grads, 1):
        ctx.adam_step(p, dev(gr, torch.float32), m, v, step, lr=1e-2, beta1=0.9, beta2=0.999, eps=1e-8)
        rp, rm, rv = R.adam(rp, gr.astype(np.float64), rm, rv, step, 1e-2, 0.9, 0.999, 1e-8)
    np.testing.assert_allclose(p.cpu().numpy(), rp, rtol=1e-5, atol=1e-6)


# --------------------------------------------------------------------------- schedules
def narrow_with(ctx, s, vf, ee, schedule, max_iter=10 ** 6):
    V0, V1, E, F = scene_dev(s)
    n = len(vf) + len(ee)
    # sentinels: a pair the schedule skipped would keep them
    hit = torch.full((n,), 255, dtype=torch.uint8, device="cuda")
    toi = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
    tmin = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    nenq = torch.full((n,), -7, dtype=torch.int64, device="cuda")
    ctx.narrow(V0, V1, E, F, dev(vf, torch.int32), dev(ee, torch.int32), DELTA, max_iter,
               out=(hit, toi, tmin, nenq), schedule=schedule)
    torch.cuda.synchronize()
    return hit.cpu().numpy(), toi.cpu().numpy(), tmin.cpu().numpy(), nenq.cpu().numpy()


def assert_identical(a, b):
    assert np.array_equal(a[0], b[0])
    assert np.array_equal(a[1].view(np.int64), b[1].view(np.int64))
    assert np.array_equal(a[2].view(np.int64), b[2].view(np.int64))
    assert np.array_equal(a[3], b[3])


def _schedule_scenes():
    yield "cloth", scenes.cloth_on_sphere(seed=7, n=32, sphere_subdivisions=2)
    yield "spheres", scenes.two_spheres()
    yield "tiny", scenes.tiny_random_scene(9, n_tris=12, extent=0.5, motion=1.0)


@pytest.mark.parametrize("max_iter", [10 ** 6, 10])
def test_every_schedule_gives_identical_outputs(ctx, max_iter):
    params, norm = random_model(6)
    for name, s in _schedule_scenes():
        V0, V1, E, F = scene_dev(s)
        vf, ee = ctx.broad(V0, V1, E, F)
        vf, ee = vf.cpu().numpy(), ee.cpu().numpy()
        n = len(vf) + len(ee)
        print(f"schedules: {name} pairs={n} max_iter={max_iter}", flush=True)
        plain = narrow_with(ctx, s, vf, ee, None, max_iter)
        assert not np.any(plain[0] == 255) and not np.any(plain[3] == -7)
        # default early wide-stage share, every pair (up to 4096) early, and none early
        for thr, mh in ((ccd.HEAVY_THRESHOLD, ccd.MAX_HEAVY), (-1e9, 4096), (0.0, 0)):
            assert_identical(plain, narrow_with(ctx, s, vf, ee, ("learned", params, norm, thr, mh), max_iter))
        rng = np.random.Generator(np.random.PCG64(n))
        assert_identical(plain, narrow_with(ctx, s, vf, ee, ("order", rng.permutation(n).astype(np.int32)),
                                            max_iter))
        assert_identical(plain, narrow_with(ctx, s, vf, ee, ("order", np.arange(n)[::-1].astype(np.int32)),
                                            max_iter))
        if name == "tiny":
            oh, ot, on_, _, omin = oracle.narrow(s.V0, s.V1, s.E, s.F, vf, ee, DELTA, max_iter)
            assert_identical(plain, (oh, ot, np.array([omin]), on_))


def test_shipped_model_gives_identical_outputs(ctx):
    try:
        params, norm, _ = sched.load_model()
    except FileNotFoundError:
        pytest.skip("no trained model file")
    s = scenes.cloth_on_sphere(seed=7, n=64, sphere_subdivisions=3)
    V0, V1, E, F = scene_dev(s)
    vf, ee = ctx.broad(V0, V1, E, F)
    vf, ee = vf.cpu().numpy(), ee.cpu().numpy()
    assert_identical(narrow_with(ctx, s, vf, ee, None), narrow_with(ctx, s, vf, ee, ("learned", params, norm)))


@pytest.mark.parametrize("bad", ["duplicate", "range", "negative"])
def test_order_schedule_rejects_non_permutation(ctx, bad):
    s = scenes.tiny_random_scene(9, n_tris=12, extent=0.5, motion=1.0)
    vf, ee = oracle.broad(s.V0, s.V1, s.E, s.F)
    n = len(vf) + len(ee)
    assert n >= 2
    perm = np.arange(n, dtype=np.int32)
    if bad == "duplicate":
        perm[1] = perm[0]
    elif bad == "range":
        perm[-1] = n
    else:
        perm[0] = -1
    with pytest.raises(ccd.CCDError) as e:
        narrow_with(ctx, s, vf, ee, ("order", perm))
    assert e.value.status == ccd.CCD_ERR_INVALID_ARG
    # the context still works
    narrow_with(ctx, s, vf, ee, ("order", np.arange(n, dtype=np.int32)))


@pytest.mark.parametrize("fill", [float("nan"), 1e30, -1e30, float("inf")])
def test_learned_schedule_with_degenerate_predictions(ctx, fill):
    """Parameters that make every prediction NaN, infinite or far out of range still give a permutation
    (each pair searched exactly once) and the plain schedule's outputs."""
    s = scenes.cloth_on_sphere(seed=7, n=32, sphere_subdivisions=2)
    V0, V1, E, F = scene_dev(s)
    vf, ee = ctx.broad(V0, V1, E, F)
    vf, ee = vf.cpu().numpy(), ee.cpu().numpy()
    params, norm = random_model(6)
    params = np.full_like(params, fill)
    plain = narrow_with(ctx, s, vf, ee, None)
    for thr, mh in ((ccd.HEAVY_THRESHOLD, ccd.MAX_HEAVY), (-1e9, 4096), (0.0, 0)):
        assert_identical(plain, narrow_with(ctx, s, vf, ee, ("learned", params, norm, thr, mh)))


def test_learned_schedule_rejects_bad_early_share(ctx):
    s = scenes.tiny_random_scene(9, n_tris=12, extent=0.5, motion=1.0)
    vf, ee = oracle.broad(s.V0, s.V1, s.E, s.F)
    params, norm = random_model(6)
    for thr, mh in ((10.0, -1), (float("nan"), 16)):
        with pytest.raises(ccd.CCDError) as e:
            narrow_with(ctx, s, vf, ee, ("learned", params, norm, thr, mh))
        assert e.value.status == ccd.CCD_ERR_INVALID_ARG


def test_learned_schedule_rejects_missing_model(ctx):
    s = scenes.tiny_random_scene(9, n_tris=4)
    V0, V1, E, F = scene_dev(s)
    vf = torch.zeros((0, 2), dtype=torch.int32, device="cuda")
    lib = ccd.load_library()
    import ctypes
    sch = ccd.Schedule(ccd.SCHED_LEARNED, None, None, None)
    tmin = torch.empty(1, dtype=torch.float64, device="cuda")
    st = lib.ccd_narrow_sched(ctx.handle, ccd._ptr(V0), ccd._ptr(V1), V0.shape[0], ccd._ptr(E), E.shape[0],
                              ccd._ptr(F), F.shape[0], None, 0, None, 0, DELTA, 10, None, None, ccd._ptr(tmin), None,
                              ctypes.byref(sch), None)
    assert st == ccd.CCD_ERR_INVALID_ARG


# --------------------------------------------------------------------------- training
def test_training_on_gpu_learns_the_cost(ctx):
    """Trained on one scene's plain-solver costs, the network ranks another scene's pairs by cost."""
    f_tr, l_tr = sched.cost_logs(ctx, scenes.cloth_on_sphere(seed=12, n=96, sphere_subdivisions=4))
    f_ev, l_ev = sched.cost_logs(ctx, scenes.cloth_on_sphere(seed=22, n=96, sphere_subdivisions=4))
    print(f"training: {f_tr.shape[0]} pairs, eval {f_ev.shape[0]} pairs", flush=True)
    params, norm, hist = sched.train(ctx, f_tr, l_tr, steps=400, batch=8192, lr=3e-3, log_every=50)
    print("minibatch mse:", hist, flush=True)
    pred = ctx.mlp_predict(params, norm, f_ev).cpu().numpy()
    lab = l_ev.cpu().numpy()
    mse0 = float(np.mean((lab - lab.mean()) ** 2))   # predicting the mean
    mse = float(np.mean((pred - lab) ** 2))
    rho = sched.spearman(pred, lab)
    print(f"held-out mse {mse:.4f} (variance {mse0:.4f}), spearman {rho:.3f}", flush=True)
    assert hist[-1][1] < hist[0][1]
    assert mse < 0.5 * mse0
    assert rho > 0.5


def test_learned_schedule_end_to_end_time(ctx):
    """What the schedule costs and buys on the benchmark's cloth scene (not one the shipped model was trained
    on), measured on the whole narrow call -- its prep with features, the network, the ordering and the early
    wide stage included -- against index order, with identical outputs.  Median over repeated calls (device
    events).  The pool alone finishes about 10 % sooner with the learned order, which the schedule's own
    passes and the early wide stage use up: end to end the two are within noise here (the median ratio has
    been measured between 0.98 and 1.034 on different GPUs of the same kind), so the test bounds the learned
    call at 5 % over the plain one and reports both ratios."""
    s = scenes.cloth_on_sphere()
    V0, V1, E, F = scene_dev(s)
    vf, ee = ctx.broad(V0, V1, E, F)
    p, nm, _ = sched.load_model()
    learned = ccd.prepare_schedule(("learned", dev(p, torch.float32), dev(nm, torch.float32), ccd.HEAVY_THRESHOLD,
                                    ccd.MAX_HEAVY))
    narrow_ms, pool_ms, outs = {"plain": [], "learned": []}, {"plain": [], "learned": []}, {}
    # alternated calls, so that clock drift affects both alike
    for it in range(43):
        for name, sc in (("plain", None), ("learned", learned)):
            out = ctx.narrow(V0, V1, E, F, vf, ee, DELTA, 10 ** 6, with_costs=True, schedule=sc)
            if it >= 3:
                st = ctx.stats()
                narrow_ms[name].append(st["narrow_ms"])
                pool_ms[name].append(st["narrow_pool_ms"])
            outs[name] = [o.cpu().numpy() for o in out]
    med = {k: float(np.median(v)) for k, v in narrow_ms.items()}
    pool = {k: float(np.median(v)) for k, v in pool_ms.items()}
    print(f"median narrow ms {med}, learned/plain {med['learned'] / med['plain']:.3f}; "
          f"pool ms {pool}, learned/plain {pool['learned'] / pool['plain']:.3f}", flush=True)
    for a, b in zip(outs["plain"], outs["learned"]):
        assert np.array_equal(a.view(np.uint8), b.view(np.uint8))
    assert med["learned"] < 1.05 * med["plain"], med
