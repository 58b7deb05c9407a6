"""Memory-budget batching of one scene (ccd_detect_budget, Sec. 5.4) against the unbatched ccd_detect, through the
C ABI: budgets small enough to split the sweep into several tile ranges (broad-phase overflow) and to re-run the
narrow phase on halves of a batch's pairs (a frontier outgrowing the buffers the budget leaves) give the same
candidate pairs, the same per-pair hit and TOI bits and the same earliest time as one unbatched call."""
import numpy as np
import pytest

import scenes

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_2112_06300_amd as ccd  # noqa: E402

DELTA = 1e-6
MB = 1 << 20


@pytest.fixture(scope="module")
def ctx():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    c = ccd.Context(0)
    yield c
    c.close()


def dev(x, dt):
    return torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dt)


def keyed(vf, ee, hit_vf, toi_vf, hit_ee, toi_ee):
    """Per-pair (hit, TOI bits) in canonical pair order."""
    ov = np.lexsort((vf[:, 1], vf[:, 0]))
    oe = np.lexsort((ee[:, 1], ee[:, 0]))
    return (vf[ov], ee[oe], hit_vf[ov], toi_vf[ov].view(np.int64), hit_ee[oe], toi_ee[oe].view(np.int64))


def unbatched(ctx, s):
    V0, V1, E, F = dev(s.V0, torch.float64), dev(s.V1, torch.float64), dev(s.E, torch.int32), dev(s.F, torch.int32)
    vf, ee = ctx.broad(V0, V1, E, F, vf_cap=8 * s.nb, ee_cap=16 * s.nb)
    hit, toi, tmin, _ = ctx.narrow(V0, V1, E, F, vf, ee, DELTA, 10 ** 6)
    n = vf.shape[0]
    h, t = hit.cpu().numpy(), toi.cpu().numpy()
    return float(tmin.cpu()[0]), keyed(vf.cpu().numpy(), ee.cpu().numpy(), h[:n], t[:n], h[n:], t[n:])


def check(ctx, s, budget, want_broad_split=True, want_narrow_split=False):
    print(f"budget {budget / MB:.0f} MiB: {s.name} nv={s.nv} ne={s.ne} nf={s.nf}", flush=True)
    tmin, ref = unbatched(ctx, s)
    V0, V1, E, F = dev(s.V0, torch.float64), dev(s.V1, torch.float64), dev(s.E, torch.int32), dev(s.F, torch.int32)
    cap_vf, cap_ee = len(ref[0]) + 16, len(ref[1]) + 16
    t, info = ctx.detect_budget(V0, V1, E, F, budget, DELTA, 10 ** 6, vf_cap=cap_vf, ee_cap=cap_ee)
    print({k: v for k, v in info.items() if not isinstance(v, np.ndarray)}, flush=True)
    assert (info["n_vf"], info["n_ee"]) == (len(ref[0]), len(ref[1]))
    got = keyed(info["vf"], info["ee"], info["vf_hit"], info["vf_toi"], info["ee_hit"], info["ee_toi"])
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
    assert np.float64(t).view(np.int64) == np.float64(tmin).view(np.int64)
    assert info["n_hits"] == int(ref[2].sum() + ref[4].sum())
    if want_broad_split:
        assert info["broad_splits"] > 0 and info["broad_batches"] > 1
    if want_narrow_split:
        assert info["narrow_splits"] > 0
    return info


def test_budget_cloth_splits_the_sweep(ctx):
    check(ctx, scenes.cloth_on_sphere(), 96 * MB)


def test_budget_gadget_torus_splits_both(ctx):
    """A 62,500-triangle perturbed torus with 300 near-degenerate gadgets, with 8,192-interval wide-stage buffers:
    the pair capacity leaves little room beside a batch's narrow workspace, and the capped gadget pairs' frontiers
    do not fit it."""
    s = scenes.perturbed_torus(seed=7, n_major=250, n_minor=125, gadgets=300)
    ctx.set_tuning({"heavy_cap_log2": 13})
    try:
        check(ctx, s, 96 * MB, want_narrow_split=True)
    finally:
        ctx.set_tuning(None)


def test_budget_large_enough_is_one_batch(ctx):
    info = check(ctx, scenes.cloth_on_sphere(n=64, sphere_subdivisions=3, seed=4), 1024 * MB, want_broad_split=False)
    assert info["broad_batches"] == 1 and info["broad_splits"] == 0 and info["narrow_splits"] == 0


def test_budget_too_small_for_the_boxes(ctx):
    s = scenes.cloth_on_sphere(n=64, sphere_subdivisions=3, seed=4)
    V0, V1, E, F = dev(s.V0, torch.float64), dev(s.V1, torch.float64), dev(s.E, torch.int32), dev(s.F, torch.int32)
    with pytest.raises(ccd.CCDError) as ei:
        ctx.detect_budget(V0, V1, E, F, 1 * MB)
    assert ei.value.status == ccd.CCD_ERR_OOM


@pytest.mark.timeout(900)
def test_budget_torus_with_gadgets(ctx):
    """The 1M-triangle torus with 12,000 gadgets (9.4M pairs) within 1.5 GiB: several sweep batches; results equal
    the unbatched call's, which the full-size test checks against the oracle."""
    from paper_2112_06300_amd import sched
    s = scenes.perturbed_torus(seed=3, gadgets=sched.TORUS_GADGETS)
    check(ctx, s, 1536 * MB)
