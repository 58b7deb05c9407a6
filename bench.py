"""Benchmark: candidate pairs per second through broad + narrow phase on one MI355X.

Workload: 256 x 256 cloth (130,050 triangles) falling onto a static 10,242-vertex
icosphere, union mesh with self and cross pairs, float64 narrow phase,
delta = 1e-6, max_iter = 1e6.  One step = ccd_detect on device-resident
V0/V1/E/F: the broad phase, then the narrow phase on its candidate pairs
(per-pair hit/TOI and the global minimum), enqueued back to back with the pair
counts passed on the device.  Inputs are seeded synthetic meshes built by
`scenes`.

The step is timed twice: with the learned schedule (features, network and
ordering inside the timed step) -- the reported value -- and with the plain
schedule (pairs in broad-phase order), reported beside it.

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
FLOPS_PER_AXIS = {0: 46, 1: 44}   # canonical evaluation sequence, per axis: VF 20 fma + 6 add, EE 16 fma + 12 add
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_cloth_on_sphere.json")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cloth-n", type=int, default=256)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (for HBM counter scaling)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the 10M-pair torus and 64-scene batch figures reported beside the main line")
    return ap.parse_args()


def source_hash(files):
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def sweep_window_tests(scene):
    """Box tests the sort-and-sweep must make on a scene (Sec. 5.2): for every query box, the candidates of the
    partner type whose lower bound on the sweep axis lies in its window, with the axis of largest centre
    variance.  Vertex windows scan faces, face windows scan vertices (strictly later lower bounds), edge
    windows scan later edges."""
    import numpy as np

    def outward(mn, mx):
        lo = mn.astype(np.float32)
        lo = np.where(lo.astype(np.float64) > mn, np.nextafter(lo, np.float32(-np.inf)), lo)
        hi = mx.astype(np.float32)
        hi = np.where(hi.astype(np.float64) < mx, np.nextafter(hi, np.float32(np.inf)), hi)
        return lo, hi

    V0, V1 = np.asarray(scene.V0), np.asarray(scene.V1)
    parts = []
    for ids in (np.arange(scene.nv)[:, None], np.asarray(scene.E), np.asarray(scene.F)):
        X = np.concatenate([V0[ids], V1[ids]], axis=1)
        parts.append(outward(X.min(axis=1), X.max(axis=1)))
    c = np.concatenate([0.5 * (lo.astype(np.float64) + hi) for lo, hi in parts])
    a = int(np.argmax(c.var(0)))
    (vl, vh), (el, eh), (fl, fh) = [(lo[:, a], hi[:, a]) for lo, hi in parts]
    vs, es, fs = np.sort(vl), np.sort(el), np.sort(fl)
    eh_sorted = eh[np.argsort(el, kind="stable")]
    w_vf = np.searchsorted(fs, vh, "right") - np.searchsorted(fs, vl, "left")
    w_fv = np.searchsorted(vs, fh, "right") - np.searchsorted(vs, fl, "right")
    w_ee = np.searchsorted(es, eh_sorted, "right") - (np.arange(len(es)) + 1)
    return int(w_vf.sum() + w_fv.sum() + np.maximum(w_ee, 0).sum())


def copy_calibration():
    import torch
    n = 1 << 28  # 2 GiB of float64 read + 2 GiB written
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 8, "copy_bytes_written": n * 8, "launches": 3}))


def cpu_baseline(scene, gpu_pairs):
    """The oracle (brute-force broad phase + sequential narrow solver) on the host cores."""
    import numpy as np
    import oracle
    nthreads = oracle.default_threads()
    t0 = time.perf_counter()
    vf, ee = oracle.broad(scene.V0, scene.V1, scene.E, scene.F, nthreads=nthreads)
    t1 = time.perf_counter()
    hit, toi, n_enq, n_eval, n_axis, tmin = oracle.narrow_with_work(scene.V0, scene.V1, scene.E, scene.F, vf, ee,
                                                                    DELTA, MAX_ITER, nthreads=nthreads)
    t2 = time.perf_counter()
    pairs = len(vf) + len(ee)
    kinds = np.concatenate([np.zeros(len(vf), np.int64), np.ones(len(ee), np.int64)])
    flops = int(np.sum(n_axis * np.where(kinds == 0, FLOPS_PER_AXIS[0], FLOPS_PER_AXIS[1])))
    return {
        "value": pairs / (t2 - t0),
        "unit": "pairs/s",
        "cores": nthreads,
        "kind": "oracle",
        "sample": f"the full workload once: brute-force broad phase ({t1 - t0:.2f} s) + narrow phase on its "
                  f"{pairs} pairs ({t2 - t1:.2f} s), {nthreads} threads",
        "pairs_match_gpu": bool(pairs == gpu_pairs),
    }, flops, int(n_eval.sum())


def extra_torus_10m(ctx, steps):
    """Narrow phase on 10M pairs drawn from the gadget torus's candidates: learned vs plain schedule."""
    import numpy as np
    import torch
    import scenes
    from paper_2112_06300_amd import sched
    s = scenes.perturbed_torus(seed=5, gadgets=sched.TORUS_GADGETS)
    dev = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dt)
    V0, V1, E, F = dev(s.V0, torch.float64), dev(s.V1, torch.float64), dev(s.E, torch.int32), dev(s.F, torch.int32)
    cvf, cee = ctx.broad(V0, V1, E, F, vf_cap=60_000_000, ee_cap=200_000_000)
    vf, ee = scenes.sample_pairs(cvf.cpu().numpy(), cee.cpu().numpy(), 10_000_000, seed=5)
    del cvf, cee
    vf, ee = dev(vf, torch.int32), dev(ee, torch.int32)
    n = vf.shape[0] + ee.shape[0]
    out = (torch.empty(n, dtype=torch.uint8, device="cuda"), torch.empty(n, dtype=torch.float64, device="cuda"),
           torch.empty(1, dtype=torch.float64, device="cuda"), None)
    try:
        params, norm, meta = sched.load_model(sched.TORUS_MODEL_PATH)
    except FileNotFoundError:
        params, norm, meta = sched.load_model()
    learned = ("learned", torch.as_tensor(params).cuda(), torch.as_tensor(norm).cuda(),
               ccd_mod().TORUS_HEAVY_THRESHOLD, ccd_mod().TORUS_MAX_HEAVY)
    res = {}
    for name, sc in (("plain", None), ("learned", learned)):
        ctx.narrow(V0, V1, E, F, vf, ee, DELTA, MAX_ITER, out=out, schedule=sc)
        ms = []
        for _ in range(steps):
            ctx.narrow(V0, V1, E, F, vf, ee, DELTA, MAX_ITER, out=out, schedule=sc)
            ms.append(ctx.stats()["narrow_ms"])
        st = ctx.stats()
        res[name] = {"narrow_ms_median": float(np.median(ms)), "pairs_per_s": n / (float(np.median(ms)) * 1e-3),
                     "pool_ms": st["narrow_pool_ms"], "heavy_ms": st["narrow_heavy_ms"],
                     "heavy_pairs": st["heavy_pairs"], "sched_heavy_pairs": st["sched_heavy_pairs"]}
    return {"workload": f"10,000,000 pairs drawn (seed 5) from the candidates of the 1M-triangle perturbed torus "
                        f"with {sched.TORUS_GADGETS} near-degenerate gadgets; narrow phase only, device events, "
                        f"median of {steps}", "model": meta.get("train"), **res,
            "learned_over_plain": res["learned"]["pairs_per_s"] / res["plain"]["pairs_per_s"]}


def extra_batch64(ctx, steps):
    """The 64-scene batch (1e3..2e5 triangles each) through one pass: captured graph vs eager launches."""
    import numpy as np
    import torch
    import scenes
    scs = scenes.scene_batch()
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


def ccd_mod():
    import paper_2112_06300_amd as ccd
    return ccd


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

    scene = scenes.cloth_on_sphere(n=args.cloth_n)
    dev = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dt)
    V0, V1 = dev(scene.V0, torch.float64), dev(scene.V1, torch.float64)
    E, F = dev(scene.E, torch.int32), dev(scene.F, torch.int32)
    ctx = ccd.Context(0)

    # size the pair buffers once (outside the timed region)
    vf0, ee0 = ctx.broad(V0, V1, E, F)
    cap_vf, cap_ee = vf0.shape[0] + 1024, ee0.shape[0] + 1024
    vf = torch.empty((cap_vf, 2), dtype=torch.int32, device="cuda")
    ee = torch.empty((cap_ee, 2), dtype=torch.int32, device="cuda")
    n_pairs_max = cap_vf + cap_ee
    hit = torch.empty(n_pairs_max, dtype=torch.uint8, device="cuda")
    toi = torch.empty(n_pairs_max, dtype=torch.float64, device="cuda")
    tmin = torch.empty(1, dtype=torch.float64, device="cuda")

    params, norm, model_meta = sched.load_model()
    learned = ccd.prepare_schedule(("learned", torch.as_tensor(params).cuda(), torch.as_tensor(norm).cuda(),
                                    ccd.HEAVY_THRESHOLD, ccd.MAX_HEAVY))

    def step(schedule):
        n_vf, n_ee = ctx.detect_into(V0, V1, E, F, vf, ee, hit, toi, tmin, None, DELTA, MAX_ITER, schedule=schedule)
        st = ctx.stats()
        return n_vf, n_ee, st, st

    extras = {}
    b_keys = ("broad_ms", "box_ms", "sort_ms", "gather_ms", "sweep_ms")
    n_keys = ("narrow_ms", "narrow_prep_ms", "narrow_sched_ms", "narrow_pool_ms", "narrow_heavy_ms",
              "heavy_pairs", "sched_heavy_pairs")

    def timed(schedule):
        for _ in range(args.warmup):
            step(schedule)
        torch.cuda.synchronize()
        acc = {k: 0.0 for k in b_keys + n_keys}
        t0 = time.perf_counter()
        for _ in range(args.steps):
            n_vf, n_ee, st_b, st_n = step(schedule)
            for k in b_keys:
                acc[k] += st_b[k]
            for k in n_keys:
                acc[k] += st_n[k]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        return n_vf, n_ee, (t1 - t0) * 1000.0 / args.steps, {k: v / args.steps for k, v in acc.items()}

    n_vf, n_ee, ms_per_step, stage = timed(learned)
    _, _, plain_ms, plain_stage = timed(None)
    K = args.steps
    pairs = n_vf + n_ee
    value = pairs / (ms_per_step / 1000.0)
    plain_value = pairs / (plain_ms / 1000.0)
    heavy_pairs = stage["heavy_pairs"]

    nv, ne, nf = scene.nv, scene.ne, scene.nf
    nb = nv + ne + nf
    # broad phase algorithmic bytes: inputs, box write, one key+id permutation, sorted record read,
    # ids for the pair filter, pair write
    broad_bytes = (48 * nv + 8 * ne + 12 * nf) + 24 * nb + 16 * nb + 28 * nb + (4 * nv + 8 * ne + 12 * nf) + 8 * pairs
    broad_gbs = broad_bytes / (stage["broad_ms"] * 1e-3) / 1e9

    if not args.no_extras:
        extras["torus_10M_pairs"] = extra_torus_10m(ctx, steps=5)
        extras["batch_64_scenes"] = extra_batch64(ctx, steps=5)

    cpu = None
    flops = None
    n_eval = None
    if not args.no_cpu_baseline:
        cpu, flops, n_eval = cpu_baseline(scene, pairs)

    search_ms = plain_stage["narrow_pool_ms"] + plain_stage["narrow_heavy_ms"]
    narrow_tflops = flops / (stage["narrow_ms"] * 1e-3) / 1e12 if flops else None
    plain_narrow_tflops = flops / (plain_stage["narrow_ms"] * 1e-3) / 1e12 if flops else None
    search_tflops = flops / (search_ms * 1e-3) / 1e12 if flops else None

    # the dominant kernel of the step (GPU event times on the library's stream)
    kernels = {"sweep_kernel": stage["sweep_ms"], "pool_kernel": stage["narrow_pool_ms"],
               "heavy_kernel": stage["narrow_heavy_ms"], "radix sort": stage["sort_ms"]}
    dominant = max(kernels, key=kernels.get)
    traffic = None
    try:
        rec = json.load(open(TRAFFIC_FILE))
        k = rec["kernels"][dominant]
        if k.get("source_hash") == source_hash(k["sources"]):
            traffic = k["bytes_per_launch"]
    except (OSError, ValueError, KeyError):
        pass
    if dominant in ("sweep_kernel", "radix sort"):
        # the sweep compares boxes: its work is the paper's window tests on this workload, 6 compares each
        tests = sweep_window_tests(scene)
        ops = tests * SWEEP_OPS_PER_TEST
        achieved = ops / (stage["sweep_ms"] * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": VALU_PEAK_TOPS, "unit": "TOP/s",
                "frac": achieved / VALU_PEAK_TOPS, "traffic": traffic, "kernel": "sweep_kernel",
                "alg_ops_per_launch": ops, "window_tests_per_launch": tests,
                "hbm_alg_bytes_per_launch": 28 * nb + (4 * nv + 8 * ne + 12 * nf) + 8 * pairs}
    else:
        # float64 vector arithmetic of the interval search: canonical flops of every pair (the oracle's
        # per-axis inclusion boxes x 46 / 44 flops), over the time of the search kernels
        roof = {"bound": "alu", "achieved": search_tflops, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": (search_tflops / FP64_PEAK_TFLOPS if search_tflops else None), "traffic": traffic,
                "kernel": "pool_kernel+heavy_kernel (interval search)", "alg_flops_per_launch": flops}

    out = {
        "metric": "candidate pairs/sec (broad+narrow, FP64, delta=1e-6), learned-sched vs plain",
        "value": value,
        "unit": "pairs/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"cloth_on_sphere: {args.cloth_n}x{args.cloth_n} cloth + 10,242-vertex icosphere "
                               f"(nv={nv}, ne={ne}, nf={nf}, boxes={nb})",
                   "pairs": pairs, "vf_pairs": n_vf, "ee_pairs": n_ee, "delta": DELTA, "max_iter": MAX_ITER,
                   "schedule": "learned", "model": model_meta.get("train"),
                   "heavy_threshold": ccd.HEAVY_THRESHOLD, "max_heavy": ccd.MAX_HEAVY},
        "plain": {"value": plain_value, "ms_per_step": plain_ms, "stages_ms": plain_stage},
        "learned_over_plain": value / plain_value,
        "roofline": roof,
        "cpu_baseline": cpu,
        "stages_ms": stage,
        "broad_hbm": {"alg_bytes": broad_bytes, "achieved_gbs": broad_gbs, "frac": broad_gbs / HBM_PEAK_GBS},
        "extras": extras,
        "narrow_fp64": {"alg_flops": flops, "canonical_evals": n_eval, "achieved_tflops": narrow_tflops,
                        "frac": (narrow_tflops / FP64_PEAK_TFLOPS if narrow_tflops else None),
                        "plain_achieved_tflops": plain_narrow_tflops,
                        "plain_search_kernels_tflops": search_tflops, "heavy_pairs": heavy_pairs,
                        "sched_heavy_pairs": stage["sched_heavy_pairs"]},
    }
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
