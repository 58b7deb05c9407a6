"""ccd_detect (broad and narrow phase in one call, pair counts passed on the
device) against the CPU oracle, through the C ABI: the same candidate pairs
and bit-identical per-pair results as oracle broad followed by oracle narrow,
for the plain and the learned schedule."""
import ctypes

import numpy as np
import pytest

import oracle
import scenes

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


def _learned():
    p, n, _ = sched.load_model()
    return ("learned", dev(p, torch.float32), dev(n, torch.float32), ccd.HEAVY_THRESHOLD, ccd.MAX_HEAVY)


def _keyed(pairs, hit, toi, nenq):
    return {tuple(int(x) for x in p): (int(h), float(t).hex(), int(e)) for p, h, t, e in zip(pairs, hit, toi, nenq)}


@pytest.mark.parametrize("scene,schedule", [
    ("cloth96", None), ("cloth96", "learned"), ("ragged", None), ("ragged", "learned"), ("spheres", "learned"),
    ("tiny", None), ("tiny", "learned"), ("cloth96", "prepared")])
def test_detect_matches_oracle(ctx, scene, schedule):
    if scene == "cloth96":
        s = scenes.cloth_on_sphere(n=96, sphere_subdivisions=3, seed=21)
    elif scene == "ragged":
        s = scenes.cloth_on_sphere(n=37, sphere_subdivisions=2, seed=5)
    elif scene == "spheres":
        s = scenes.two_spheres()
    else:
        s = scenes.tiny_random_scene(11)
    print(f"detect parity: {s.name} nv={s.nv} schedule={schedule}", flush=True)
    V0, V1, E, F = dev(s.V0, torch.float64), dev(s.V1, torch.float64), dev(s.E, torch.int32), dev(s.F, torch.int32)
    ovf, oee = oracle.broad(s.V0, s.V1, s.E, s.F)
    cap_vf, cap_ee = len(ovf) + 100, len(oee) + 77  # ragged capacities, larger than needed
    vf = torch.full((cap_vf, 2), -1, dtype=torch.int32, device="cuda")
    ee = torch.full((cap_ee, 2), -1, dtype=torch.int32, device="cuda")
    n = cap_vf + cap_ee
    hit = torch.empty(n, dtype=torch.uint8, device="cuda")
    toi = torch.empty(n, dtype=torch.float64, device="cuda")
    tmin = torch.empty(1, dtype=torch.float64, device="cuda")
    nenq = torch.empty(n, dtype=torch.int64, device="cuda")
    sc = _learned() if schedule == "learned" else None
    if schedule == "prepared":
        sc = ccd.prepare_schedule(_learned())
    n_vf, n_ee = ctx.detect_into(V0, V1, E, F, vf, ee, hit, toi, tmin, nenq, DELTA, 10 ** 6, schedule=sc)
    torch.cuda.synchronize()
    assert (n_vf, n_ee) == (len(ovf), len(oee))
    gvf, gee = vf[:n_vf].cpu().numpy(), ee[:n_ee].cpu().numpy()
    h, t, e = hit.cpu().numpy(), toi.cpu().numpy(), nenq.cpu().numpy()
    oh, ot, on_, _, omin = oracle.narrow(s.V0, s.V1, s.E, s.F, ovf, oee, DELTA)
    assert _keyed(gvf, h[:n_vf], t[:n_vf], e[:n_vf]) == _keyed(ovf, oh[:len(ovf)], ot[:len(ovf)], on_[:len(ovf)])
    m = n_vf + n_ee
    assert _keyed(gee, h[n_vf:m], t[n_vf:m], e[n_vf:m]) == _keyed(oee, oh[len(ovf):], ot[len(ovf):], on_[len(ovf):])
    assert np.float64(tmin.cpu()[0]).view(np.int64) == np.float64(omin).view(np.int64)
    st = ctx.stats()
    assert st["broad_ms"] > 0 and st["narrow_ms"] > 0


def test_detect_capacity_error_reports_counts(ctx):
    s = scenes.cloth_on_sphere(n=40, sphere_subdivisions=2, seed=7)
    ovf, oee = oracle.broad(s.V0, s.V1, s.E, s.F)
    assert len(ovf) > 10 and len(oee) > 10
    V0, V1, E, F = dev(s.V0, torch.float64), dev(s.V1, torch.float64), dev(s.E, torch.int32), dev(s.F, torch.int32)
    lib = ccd.load_library()
    cap_vf, cap_ee = len(ovf) // 2, len(oee)
    vf = torch.empty((cap_vf, 2), dtype=torch.int32, device="cuda")
    ee = torch.empty((cap_ee, 2), dtype=torch.int32, device="cuda")
    hit = torch.empty(cap_vf + cap_ee, dtype=torch.uint8, device="cuda")
    toi = torch.empty(cap_vf + cap_ee, dtype=torch.float64, device="cuda")
    tmin = torch.empty(1, dtype=torch.float64, device="cuda")
    n_vf, n_ee = ctypes.c_int64(), ctypes.c_int64()
    p = lambda t: ctypes.c_void_p(t.data_ptr())
    st = lib.ccd_detect(ctx.handle, p(V0), p(V1), V0.shape[0], p(E), E.shape[0], p(F), F.shape[0], p(vf), cap_vf,
                        ctypes.byref(n_vf), p(ee), cap_ee, ctypes.byref(n_ee), DELTA, 10 ** 6, p(hit), p(toi),
                        p(tmin), None, None, None)
    assert st == ccd.CCD_ERR_CAPACITY
    assert (n_vf.value, n_ee.value) == (len(ovf), len(oee))
    with pytest.raises(ccd.CCDError):
        ctx.detect_into(V0, V1, E, F, vf, ee, hit, toi, tmin)


def test_detect_rejects_order_schedule(ctx):
    s = scenes.cloth_on_sphere(n=16, sphere_subdivisions=1, seed=3)
    V0, V1, E, F = dev(s.V0, torch.float64), dev(s.V1, torch.float64), dev(s.E, torch.int32), dev(s.F, torch.int32)
    vf = torch.empty((4096, 2), dtype=torch.int32, device="cuda")
    ee = torch.empty((4096, 2), dtype=torch.int32, device="cuda")
    hit = torch.empty(8192, dtype=torch.uint8, device="cuda")
    toi = torch.empty(8192, dtype=torch.float64, device="cuda")
    tmin = torch.empty(1, dtype=torch.float64, device="cuda")
    perm = torch.arange(8192, dtype=torch.int32, device="cuda")
    with pytest.raises(ccd.CCDError, match="INVALID_ARG"):
        ctx.detect_into(V0, V1, E, F, vf, ee, hit, toi, tmin, schedule=("order", perm))


def test_context_created_before_torch_touches_the_gpu():
    """A fresh process that creates a context before torch has used the GPU, then hands torch tensors to it:
    the library and torch share one HIP runtime, so both see the GPU and the call matches the oracle."""
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    code = (
        "import numpy as np\n"
        "import paper_2112_06300_amd as ccd\n"
        "import oracle, scenes\n"
        "c = ccd.Context(0)\n"
        "import torch\n"
        "s = scenes.tiny_random_scene(3, n_tris=40, extent=1.0, motion=0.5)\n"
        "d = lambda x, t: torch.as_tensor(np.ascontiguousarray(x)).to('cuda', t)\n"
        "vf, ee = c.broad(d(s.V0, torch.float64), d(s.V1, torch.float64), d(s.E, torch.int32), d(s.F, torch.int32))\n"
        "canon = lambda p: p[np.lexsort((p[:, 1], p[:, 0]))] if len(p) else p\n"
        "ovf, oee = oracle.broad(s.V0, s.V1, s.E, s.F)\n"
        "assert np.array_equal(canon(vf.cpu().numpy()), ovf) and np.array_equal(canon(ee.cpu().numpy()), oee)\n"
        "c.close()\n"
        "print('ok', len(ovf), len(oee))\n")
    env = dict(os.environ)
    env["PYTHONPATH"] = root + os.pathsep + env.get("PYTHONPATH", "")
    print("child: context before torch", flush=True)
    r = subprocess.run([sys.executable, "-c", code], cwd=root, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
    assert r.stdout.strip().splitlines()[-1].startswith("ok")
