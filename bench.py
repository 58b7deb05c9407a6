"""Benchmark: candidate pairs per second through broad + narrow phase on one MI355X.

Workload: the 1M-triangle randomly perturbed torus (500k vertices, 1.5M edges,
1M faces; t = 0 perturbation N(0, (0.1 e)^2), displacement N(0, (0.5 e)^2))
with 12,000 near-degenerate two-triangle gadgets inside the tube (parallel
sliding edges and grazing vertex-face contacts at separations 0, 1e-12 e and
1e-9 e, about 1 % of the candidate pairs), self collision, float64 narrow
phase, delta = 1e-6, max_iter = 1e6.  One step = ccd_detect on
device-resident V0/V1/E/F: the broad phase, then the narrow phase on its
candidate pairs (per-pair hit/TOI and the global minimum), enqueued back to
back with the pair counts passed on the device.  Inputs are seeded synthetic
meshes built by `scenes`.

The step is timed with the learned schedule (features, network and ordering
inside the timed step) -- the reported value -- and with the plain schedule
(pairs in broad-phase order); their ratio comes from steps of the two
alternated, median and spread.  Beside them: the narrow phase on the same
pairs with a random and a true-cost order placed the way the learned schedule
places pairs (the references the learned one is judged by), Alg. 3's single
shared t* (only the earliest time), and the other workloads (cloth on sphere,
10M sampled torus pairs, the 64-scene batch of large and of small scenes, all pairs of two
spheres).

Prints one JSON line.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6      # MI355X FP64 vector (FMA = 2 flops)
VALU_PEAK_TOPS = 39.3        # MI355X vector ALU, one 32-bit op per lane per cycle: 256 CU x 4 SIMD x 16 lanes x 2.4 GHz
SWEEP_OPS_PER_TEST = 6       # sweep box test: upper key, window-order key and four bound compares
DELTA = 1e-6
MAX_ITER = 10 ** 6
# canonical float64 flops per interval evaluation (8 corners x 3 axes of the fixed sequence):
# vertex-face 20 fma + 6 add per axis, edge-edge 16 fma + 12 add per axis, fma = 2
FLOPS_PER_EVAL = {"vf": 138, "ee": 132}
TORUS_SEED, TORUS_GADGETS = 3, 12000
MANIFEST = os.path.join(ROOT, "tests", "golden", "torus_gadgets_manifest.json")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_torus_gadgets.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (for HBM counter scaling)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the figures reported beside the main line (orderings, shared t*, other workloads)")
    ap.add_argument("--profile-steps", type=int, default=0,
                    help="only run this many plain and learned steps of the main workload (for profilers)")
    ap.add_argument("--profile-workload", choices=("torus", "cloth"), default="torus",
                    help="workload of --profile-steps: the gadget torus, or the 256 x 256 cloth on a sphere")
    return ap.parse_args()


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def scene_hash(s):
    import numpy as np
    h = hashlib.sha256()
    for a, dt in ((s.V0, np.float64), (s.V1, np.float64), (s.E, np.int32), (s.F, np.int32)):
        h.update(np.ascontiguousarray(a, dtype=dt).tobytes())
    return h.hexdigest()


def copy_calibration():
    import torch
    n = 1 << 28  # 2 GiB of float64 read + 2 GiB written
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}))


def cpu_baseline(scene, pairs, vf, ee, rng_seed=1):
    """The oracle on a bounded sample of the workload, scaled to the whole: its brute-force broad phase over
    1/64 of the rows (rate of box tests, times all tests) and its narrow phase on 1/16 of the pairs drawn
    uniformly (seeded), times 16."""
    import numpy as np
    import oracle
    nthreads = oracle.default_threads()
    stride = 64
    t0 = time.perf_counter()
    _, _, tvf, tee = oracle.broad_sample(scene.V0, scene.V1, scene.E, scene.F, stride, nthreads=nthreads)
    t1 = time.perf_counter()
    all_tests = scene.nv * scene.nf + scene.ne * (scene.ne - 1) / 2
    broad_s = (t1 - t0) * all_tests / (tvf + tee)
    rng = np.random.Generator(np.random.PCG64(rng_seed))
    keep = rng.random(len(vf) + len(ee)) < 1.0 / 16
    svf, see = vf[keep[:len(vf)]], ee[keep[len(vf):]]
    t2 = time.perf_counter()
    oracle.narrow(scene.V0, scene.V1, scene.E, scene.F, svf, see, DELTA, MAX_ITER, nthreads=nthreads)
    t3 = time.perf_counter()
    narrow_s = (t3 - t2) * (len(vf) + len(ee)) / max(1, len(svf) + len(see))
    return {
        "value": pairs / (broad_s + narrow_s),
        "unit": "pairs/s",
        "cores": nthreads,
        "kind": "oracle",
        "sample": (f"brute-force broad phase over 1/{stride} of its rows ({(tvf + tee):.3g} of {all_tests:.3g} box "
                   f"tests in {t1 - t0:.1f} s, scaled: {broad_s:.0f} s) + narrow phase on {len(svf) + len(see)} "
                   f"uniformly drawn pairs of {len(vf) + len(ee)} ({t3 - t2:.1f} s, scaled: {narrow_s:.1f} s), "
                   f"{nthreads} threads"),
    }


def read_manifest(scene):
    """The oracle's canonical work on the torus workload (written by tests/golden/make_torus_manifest.py), if
    it was computed for exactly these inputs."""
    try:
        man = json.load(open(MANIFEST))
    except (OSError, ValueError):
        return None
    return man if man.get("input_sha256") == scene_hash(scene) else None


def ccd_mod():
    import paper_2112_06300_amd as ccd
    return ccd


class Workload:
    """A scene on the device with pair and result buffers sized once (outside any timed region)."""

    def __init__(self, ctx, scene, slack=1024):
        import numpy as np
        import torch
        self.ctx, self.scene = ctx, scene
        dev = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dt)
        self.V0, self.V1 = dev(scene.V0, torch.float64), dev(scene.V1, torch.float64)
        self.E, self.F = dev(scene.E, torch.int32), dev(scene.F, torch.int32)
        vf0, ee0 = ctx.broad(self.V0, self.V1, self.E, self.F, vf_cap=4 * scene.nb, ee_cap=8 * scene.nb)
        self.cap_vf, self.cap_ee = vf0.shape[0] + slack, ee0.shape[0] + slack
        del vf0, ee0
        self.vf = torch.empty((self.cap_vf, 2), dtype=torch.int32, device="cuda")
        self.ee = torch.empty((self.cap_ee, 2), dtype=torch.int32, device="cuda")
        n = self.cap_vf + self.cap_ee
        self.hit = torch.empty(n, dtype=torch.uint8, device="cuda")
        self.toi = torch.empty(n, dtype=torch.float64, device="cuda")
        self.tmin = torch.empty(1, dtype=torch.float64, device="cuda")
        self.n_vf = self.n_ee = 0

    def step(self, schedule=None, options=None):
        self.n_vf, self.n_ee = self.ctx.detect_into(self.V0, self.V1, self.E, self.F, self.vf, self.ee, self.hit,
                                                    self.toi, self.tmin, None, DELTA, MAX_ITER, schedule=schedule,
                                                    options=options)
        return self.n_vf + self.n_ee

    def pairs(self):
        return self.vf[:self.n_vf].clone(), self.ee[:self.n_ee].clone()


B_KEYS = ("broad_ms", "box_ms", "sort_ms", "gather_ms", "sweep_ms")
N_KEYS = ("narrow_ms", "narrow_prep_ms", "narrow_sched_ms", "narrow_pool_ms", "narrow_heavy_ms", "heavy_pairs",
          "sched_heavy_pairs", "heavy_reruns")


def timed_steps(w, schedule, steps, warmup, options=None):
    """W untimed steps, then exactly K steps bracketed by device synchronizations: (ms per step, mean stage times)."""
    import torch
    for _ in range(warmup):
        w.step(schedule, options)
    torch.cuda.synchronize()
    acc = {k: 0.0 for k in B_KEYS + N_KEYS}
    t0 = time.perf_counter()
    for _ in range(steps):
        w.step(schedule, options)
        st = w.ctx.stats()
        for k in acc:
            acc[k] += st[k]
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return (t1 - t0) * 1000.0 / steps, {k: v / steps for k, v in acc.items()}


def alternated(w, a, b, rounds, options=None):
    """Steps of schedules a and b alternated (a first in even rounds, b first in odd ones): per-step wall times."""
    import numpy as np
    import torch
    ta, tb = [], []
    for r in range(rounds):
        for which in ((0, 1) if r % 2 == 0 else (1, 0)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            w.step(a if which == 0 else b, options)
            t1 = time.perf_counter()
            (ta if which == 0 else tb).append((t1 - t0) * 1000.0)
    ta, tb = np.array(ta), np.array(tb)
    ratio = tb / ta  # per round: b's time over a's, i.e. a's speed-up over b
    return {"a_ms_median": float(np.median(ta)), "b_ms_median": float(np.median(tb)),
            "speedup_median": float(np.median(ratio)),
            "speedup_p25_p75": [float(np.percentile(ratio, 25)), float(np.percentile(ratio, 75))],
            "rounds": rounds}


def orderings(w, learned, rounds=5):
    """The narrow phase alone on the workload's pairs with plain, learned, random-cost and true-cost placement
    (the last two place pairs exactly as the learned schedule does, from random values and from the plain
    solver's own log2(1 + n_enq)): median device time of `rounds` runs of each, interleaved."""
    import numpy as np
    import torch
    ctx = w.ctx
    vf, ee = w.pairs()
    n = vf.shape[0] + ee.shape[0]
    out = (torch.empty(n, dtype=torch.uint8, device="cuda"), torch.empty(n, dtype=torch.float64, device="cuda"),
           torch.empty(1, dtype=torch.float64, device="cuda"), torch.empty(n, dtype=torch.int64, device="cuda"))
    ctx.narrow(w.V0, w.V1, w.E, w.F, vf, ee, DELTA, MAX_ITER, out=out)
    true_cost = torch.log2(1.0 + out[3].to(torch.float32))
    ref_hit, ref_toi = out[0].clone(), out[1].clone()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(7)
    rand_cost = torch.rand(n, generator=gen, device="cuda", dtype=torch.float32) * float(true_cost.max().item())
    ccd = ccd_mod()
    thr, mh = learned.sch.heavy_threshold, learned.sch.max_heavy
    kinds = {"plain": None, "learned": learned,
             "random_cost": ccd.prepare_schedule(("cost", rand_cost, thr, mh)),
             "true_cost": ccd.prepare_schedule(("cost", true_cost, thr, mh))}
    ms = {k: [] for k in kinds}
    same = True
    for r in range(rounds):
        for k, sc in kinds.items():
            ctx.narrow(w.V0, w.V1, w.E, w.F, vf, ee, DELTA, MAX_ITER, out=out, schedule=sc)
            ms[k].append(ctx.stats()["narrow_ms"])
            if r == 0:
                same = same and bool(torch.equal(out[0], ref_hit)) and bool(torch.equal(out[1], ref_toi))
    med = {k: float(np.median(v)) for k, v in ms.items()}
    return {"pairs": int(n), "narrow_ms_median": med,
            "speedup_over_plain": {k: med["plain"] / v for k, v in med.items()},
            "outputs_identical": same, "rounds": rounds,
            "note": "narrow phase only; learned includes its features, network and ordering passes"}


def earliest_only(w, steps):
    """Alg. 3's single shared t* (only the earliest time defined) against the per-pair mode: whole step."""
    import torch
    opts = {"earliest_only": 1}
    ms_g, st_g = timed_steps(w, None, steps, 2, options=opts)
    tg = float(w.tmin.cpu()[0])
    ms_p, _ = timed_steps(w, None, steps, 2)
    tp = float(w.tmin.cpu()[0])
    pairs = w.n_vf + w.n_ee
    return {"earliest_only_ms_per_step": ms_g, "per_pair_ms_per_step": ms_p,
            "earliest_only_pairs_per_s": pairs / (ms_g * 1e-3), "per_pair_pairs_per_s": pairs / (ms_p * 1e-3),
            "toi_min_earliest_only": tg, "toi_min_per_pair": tp, "narrow_ms_earliest_only": st_g["narrow_ms"]}


def extra_cloth(ctx, steps):
    """The 256 x 256 cloth on a 10,242-vertex sphere: learned (its own model) vs plain, whole step."""
    import scenes
    from paper_2112_06300_amd import sched
    ccd = ccd_mod()
    w = Workload(ctx, scenes.cloth_on_sphere(n=256))
    params, norm, meta = sched.load_model(sched.MODEL_PATH)
    import torch
    learned = ccd.prepare_schedule(("learned", torch.as_tensor(params).cuda(), torch.as_tensor(norm).cuda(),
                                    ccd.HEAVY_THRESHOLD, ccd.MAX_HEAVY))
    ms_l, st_l = timed_steps(w, learned, steps, 3)
    ms_p, st_p = timed_steps(w, None, steps, 3)
    cmp_ = alternated(w, learned, None, 10)
    pairs = w.n_vf + w.n_ee
    return {"workload": "cloth_on_sphere: 256x256 cloth + 10,242-vertex icosphere", "pairs": pairs,
            "learned_pairs_per_s": pairs / (ms_l * 1e-3), "plain_pairs_per_s": pairs / (ms_p * 1e-3),
            "learned_ms": ms_l, "plain_ms": ms_p, "learned_over_plain_alternated": cmp_,
            "learned_stages_ms": st_l, "plain_stages_ms": st_p, "earliest_only": earliest_only(w, steps)}


def extra_torus_10m(ctx, steps):
    """Narrow phase on 10M pairs drawn from the gadget torus's candidates: learned vs plain schedule."""
    import numpy as np
    import torch
    import scenes
    from paper_2112_06300_amd import sched
    s = scenes.perturbed_torus(seed=5, gadgets=TORUS_GADGETS)
    dev = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dt)
    V0, V1, E, F = dev(s.V0, torch.float64), dev(s.V1, torch.float64), dev(s.E, torch.int32), dev(s.F, torch.int32)
    cvf, cee = ctx.broad(V0, V1, E, F, vf_cap=60_000_000, ee_cap=200_000_000)
    vf, ee = scenes.sample_pairs(cvf.cpu().numpy(), cee.cpu().numpy(), 10_000_000, seed=5)
    del cvf, cee
    vf, ee = dev(vf, torch.int32), dev(ee, torch.int32)
    n = vf.shape[0] + ee.shape[0]
    out = (torch.empty(n, dtype=torch.uint8, device="cuda"), torch.empty(n, dtype=torch.float64, device="cuda"),
           torch.empty(1, dtype=torch.float64, device="cuda"), None)
    params, norm, meta = sched.load_model(sched.TORUS_MODEL_PATH)
    learned = ccd_mod().prepare_schedule(("learned", torch.as_tensor(params).cuda(), torch.as_tensor(norm).cuda(),
                                          ccd_mod().TORUS_HEAVY_THRESHOLD, ccd_mod().TORUS_MAX_HEAVY))
    ms = {"plain": [], "learned": []}
    for name, sc in (("plain", None), ("learned", learned)):
        ctx.narrow(V0, V1, E, F, vf, ee, DELTA, MAX_ITER, out=out, schedule=sc)
    for _ in range(steps):
        for name, sc in (("plain", None), ("learned", learned)):
            ctx.narrow(V0, V1, E, F, vf, ee, DELTA, MAX_ITER, out=out, schedule=sc)
            ms[name].append(ctx.stats()["narrow_ms"])
    res = {k: {"narrow_ms_median": float(np.median(v)), "pairs_per_s": n / (float(np.median(v)) * 1e-3)}
           for k, v in ms.items()}
    return {"workload": f"10,000,000 pairs drawn (seed 5) from the candidates of the 1M-triangle perturbed torus "
                        f"with {TORUS_GADGETS} near-degenerate gadgets; narrow phase only, device events, "
                        f"median of {steps} alternated", "model": meta.get("train"), **res,
            "learned_over_plain": res["learned"]["pairs_per_s"] / res["plain"]["pairs_per_s"]}


def extra_batch64(ctx, steps, small=False):
    """The 64-scene batch (1e3..2e5 triangles each; small: 1e2..2e3) through one pass: captured graph vs
    eager launches."""
    import numpy as np
    import torch
    import scenes
    scs = scenes.scene_batch(t_min=1e2, t_max=2e3) if small else scenes.scene_batch()
    V0, V1, E, F, vo, eo, fo = scenes.concat_scenes(scs)
    nb = int(vo[-1] + eo[-1] + fo[-1])
    b = ccd_mod().Batch(ctx, vo, eo, fo, 3 * nb, 6 * nb)
    dev = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dt)
    inp = (dev(V0, torch.float64), dev(V1, torch.float64), dev(E, torch.int32), dev(F, torch.int32))
    res = {}
    for name, g in (("eager", False), ("graph", True)):
        b.run(*inp, DELTA, MAX_ITER, use_graph=g)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            b.run(*inp, DELTA, MAX_ITER, use_graph=g)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1000.0 / steps
        res[name] = {"ms_per_pass": ms, "pairs_per_s": (b.n_vf + b.n_ee) / (ms * 1e-3)}
    out = {"workload": f"64 scenes, {int(fo[-1])} triangles, {nb} boxes, CSR layout, broad + narrow in one pass",
           "pairs": b.n_vf + b.n_ee, **res}
    b.close()
    return out


def extra_two_spheres_all_pairs(ctx, steps):
    """Every VF and EE pair of the two jittered icospheres (10,631,100 queries, about one evaluation each)."""
    import numpy as np
    import torch
    import oracle
    import scenes
    s = scenes.two_spheres()
    vf, ee = oracle.all_pairs(s.E, s.F, s.nv)
    dev = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dt)
    V0, V1, E, F = dev(s.V0, torch.float64), dev(s.V1, torch.float64), dev(s.E, torch.int32), dev(s.F, torch.int32)
    vf, ee = dev(vf, torch.int32), dev(ee, torch.int32)
    n = vf.shape[0] + ee.shape[0]
    out = (torch.empty(n, dtype=torch.uint8, device="cuda"), torch.empty(n, dtype=torch.float64, device="cuda"),
           torch.empty(1, dtype=torch.float64, device="cuda"), None)
    ctx.narrow(V0, V1, E, F, vf, ee, DELTA, MAX_ITER, out=out)
    ms = []
    for _ in range(steps):
        ctx.narrow(V0, V1, E, F, vf, ee, DELTA, MAX_ITER, out=out)
        ms.append(ctx.stats()["narrow_ms"])
    med = float(np.median(ms))
    return {"workload": "two icospheres (642 vertices each), all 10,631,100 VF + EE pairs, narrow phase only",
            "narrow_ms_median": med, "pairs_per_s": n / (med * 1e-3)}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the narrow and broad phases of this "
              "library run on a single MI355X; sharding across GPUs is designed but not built.",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calibration:
        copy_calibration()
        return
    import numpy as np
    import scenes
    import paper_2112_06300_amd as ccd
    from paper_2112_06300_amd import sched

    if args.profile_steps and args.profile_workload == "cloth":
        log("building the cloth workload")
        ctx = ccd.Context(0)
        w = Workload(ctx, scenes.cloth_on_sphere(n=256))
        params, norm, model_meta = sched.load_model(sched.MODEL_PATH)
        learned = ccd.prepare_schedule(("learned", torch.as_tensor(params).cuda(), torch.as_tensor(norm).cuda(),
                                        ccd.HEAVY_THRESHOLD, ccd.MAX_HEAVY))
    else:
        log("building the torus workload")
        scene = scenes.perturbed_torus(seed=TORUS_SEED, gadgets=TORUS_GADGETS)
        ctx = ccd.Context(0)
        w = Workload(ctx, scene)
        params, norm, model_meta = sched.load_model(sched.TORUS_MODEL_PATH)
        learned = ccd.prepare_schedule(("learned", torch.as_tensor(params).cuda(), torch.as_tensor(norm).cuda(),
                                        ccd.TORUS_HEAVY_THRESHOLD, ccd.TORUS_MAX_HEAVY))
    if args.profile_steps:
        for _ in range(args.profile_steps):
            w.step(None)
            w.step(learned)
        torch.cuda.synchronize()
        log(f"profile steps done: {w.n_vf + w.n_ee} pairs")
        ctx.close()
        return

    log("timing learned steps")
    ms_per_step, stage = timed_steps(w, learned, args.steps, args.warmup)
    pairs = w.n_vf + w.n_ee
    n_vf, n_ee = w.n_vf, w.n_ee
    tmin_learned = float(w.tmin.cpu()[0])
    log("timing plain steps")
    plain_ms, plain_stage = timed_steps(w, None, args.steps, args.warmup)
    tmin_plain = float(w.tmin.cpu()[0])
    log("alternating learned and plain steps")
    cmp_ = alternated(w, learned, None, max(6, args.steps // 2))
    value = pairs / (ms_per_step / 1000.0)
    plain_value = pairs / (plain_ms / 1000.0)

    nv, ne, nf = scene.nv, scene.ne, scene.nf
    nb = nv + ne + nf
    # broad phase algorithmic bytes: inputs, box write, one key+id permutation, sorted record read,
    # ids for the pair filter, pair write
    broad_bytes = (48 * nv + 8 * ne + 12 * nf) + 24 * nb + 16 * nb + 28 * nb + (4 * nv + 8 * ne + 12 * nf) + 8 * pairs
    broad_gbs = broad_bytes / (stage["broad_ms"] * 1e-3) / 1e9

    man = read_manifest(scene)
    flops = None
    n_eval = None
    if man and man["n_vf"] == n_vf and man["n_ee"] == n_ee:
        n_eval = man["n_eval"]["vf"] + man["n_eval"]["ee"]
        flops = man["n_eval"]["vf"] * FLOPS_PER_EVAL["vf"] + man["n_eval"]["ee"] * FLOPS_PER_EVAL["ee"]

    extras = {}
    if not args.no_extras:
        log("orderings")
        extras["orderings_torus"] = orderings(w, learned)
        log("earliest-only mode")
        extras["earliest_only_torus"] = earliest_only(w, 5)
        log("cloth")
        extras["cloth_on_sphere"] = extra_cloth(ctx, 10)
        log("10M torus pairs")
        extras["torus_10M_pairs"] = extra_torus_10m(ctx, steps=5)
        log("64-scene batch")
        extras["batch_64_scenes"] = extra_batch64(ctx, steps=5)
        log("64 small scenes")
        extras["batch_64_small_scenes"] = extra_batch64(ctx, steps=50, small=True)
        log("two spheres, all pairs")
        extras["two_spheres_all_pairs"] = extra_two_spheres_all_pairs(ctx, steps=5)

    cpu = None
    if not args.no_cpu_baseline:
        log("oracle sample on the host")
        cvf, cee = w.pairs()
        cpu = cpu_baseline(scene, pairs, cvf.cpu().numpy(), cee.cpu().numpy())
    ctx.close()

    # the dominant kernel of the step (GPU event times on the library's stream)
    kernels = {"sweep_kernel": stage["sweep_ms"], "pool_kernel": stage["narrow_pool_ms"],
               "heavy_kernel": stage["narrow_heavy_ms"], "radix sort": stage["sort_ms"]}
    dominant = max(kernels, key=kernels.get)
    traffic = None
    try:
        rec = json.load(open(TRAFFIC_FILE))
        k = rec["kernels"]["pool_kernel+heavy_kernel" if dominant in ("pool_kernel", "heavy_kernel") else dominant]
        if k.get("source_hash") == source_hash(k["sources"]):
            traffic = k["bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        pass
    # float64 vector arithmetic of the interval search: the canonical flops of every pair (the oracle's
    # interval evaluations x 138 / 132 flops), over the time of the search kernels of the plain step
    search_ms = plain_stage["narrow_pool_ms"] + plain_stage["narrow_heavy_ms"]
    search_tflops = flops / (search_ms * 1e-3) / 1e12 if flops else None
    if dominant in ("sweep_kernel", "radix sort"):
        roof = {"bound": "hbm", "achieved": broad_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": broad_gbs / HBM_PEAK_GBS, "traffic": traffic, "kernel": "broad phase",
                "alg_bytes_per_launch": broad_bytes}
    else:
        roof = {"bound": "alu", "achieved": search_tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": (search_tflops / FP64_PEAK_TFLOPS if search_tflops else None), "traffic": traffic,
                "kernel": "pool_kernel+heavy_kernel (interval search, plain step)",
                "alg_flops_per_launch": flops, "canonical_evals": n_eval, "search_ms": search_ms,
                "flop_source": "tests/golden/torus_gadgets_manifest.json" if flops else None}

    out = {
        "metric": "candidate pairs/sec (broad+narrow, FP64, delta=1e-6), learned-sched vs plain",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"perturbed_torus with near-degenerate gadgets: 1M-triangle torus (R=1, r=0.4, "
                               f"1000x500 grid) + {TORUS_GADGETS} gadgets, seed {TORUS_SEED} (nv={nv}, ne={ne}, "
                               f"nf={nf}, boxes={nb})",
                   "pairs": pairs, "vf_pairs": n_vf, "ee_pairs": n_ee, "delta": DELTA, "max_iter": MAX_ITER,
                   "schedule": "learned", "model": model_meta.get("train"),
                   "heavy_threshold": ccd.TORUS_HEAVY_THRESHOLD, "max_heavy": ccd.TORUS_MAX_HEAVY},
        "plain": {"value": plain_value, "ms_per_step": plain_ms, "stages_ms": plain_stage},
        "learned_over_plain": value / plain_value,
        "learned_over_plain_alternated": cmp_,
        "roofline": roof,
        "cpu_baseline": cpu,
        "stages_ms": stage,
        "dominant_kernel": dominant,
        "toi_min": {"learned": tmin_learned, "plain": tmin_plain,
                    "oracle": man["toi_min"] if man else None},
        "broad_hbm": {"alg_bytes": broad_bytes, "achieved_gbs": broad_gbs, "frac": broad_gbs / HBM_PEAK_GBS},
        "narrow_fp64": {"alg_flops": flops, "canonical_evals": n_eval,
                        "learned_narrow_tflops": flops / (stage["narrow_ms"] * 1e-3) / 1e12 if flops else None,
                        "plain_narrow_tflops": flops / (plain_stage["narrow_ms"] * 1e-3) / 1e12 if flops else None,
                        "plain_search_kernels_tflops": search_tflops},
        "extras": extras,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
