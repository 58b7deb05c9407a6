"""Write torus_gadgets_manifest.json: the oracle's answer on the 1M-triangle perturbed torus with 12,000
near-degenerate gadgets (seed 3), the largest single-GPU workload.

Calls only the oracle (brute-force broad phase, per-pair narrow phase; Sec. 5.5: brute force defines the pair
set) and the seeded scene generator.  The oracle takes tens of minutes on 8 cores, so the full-size GPU test
and the benchmark read this file instead, guarded by a hash of the scene's arrays (a changed generator makes
them fall back or report no figure).  Stored:
  - the input hash and sizes, the pair counts and a hash of the canonically sorted pairs;
  - a hash of the per-pair results (hit, TOI bits, n_enq) in canonical pair order, and one of hit and TOI
    bits alone;
  - the earliest time of impact (bits), the number of capped pairs and whether the earliest is a capped one;
  - the canonical work: interval evaluations and per-axis inclusion boxes by pair kind (the benchmark's
    flop count), and a histogram of evaluations per pair.

Usage: python tests/golden/make_torus_manifest.py [--threads N]
"""
import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import scenes  # noqa: E402

OUT = os.path.join(HERE, "torus_gadgets_manifest.json")
SEED, GADGETS = 3, 12000
DELTA, MAX_ITER = 1e-6, 10 ** 6


def scene_hash(s):
    h = hashlib.sha256()
    for a, dt in ((s.V0, np.float64), (s.V1, np.float64), (s.E, np.int32), (s.F, np.int32)):
        h.update(np.ascontiguousarray(a, dtype=dt).tobytes())
    return h.hexdigest()


def canonical_order(vf, ee):
    """Index permutations sorting VF and EE pairs lexicographically."""
    return np.lexsort((vf[:, 1], vf[:, 0])), np.lexsort((ee[:, 1], ee[:, 0]))


def pairs_hash(vf, ee):
    """sha256 of the sorted VF pairs then the sorted EE pairs (int32)."""
    ov, oe = canonical_order(vf, ee)
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(vf[ov], np.int32).tobytes())
    h.update(np.ascontiguousarray(ee[oe], np.int32).tobytes())
    return h.hexdigest()


def results_hash(vf, ee, hit, toi, n_enq):
    """sha256 of hit (uint8), TOI bits (float64) and n_enq (int64), each in canonical pair order."""
    ov, oe = canonical_order(vf, ee)
    perm = np.concatenate([ov, len(vf) + oe])
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(hit[perm], np.uint8).tobytes())
    h.update(np.ascontiguousarray(toi[perm], np.float64).tobytes())
    h.update(np.ascontiguousarray(n_enq[perm], np.int64).tobytes())
    return h.hexdigest()


def hit_toi_hash(vf, ee, hit, toi):
    """sha256 of hit (uint8) and TOI bits (float64) in canonical pair order (for callers without n_enq)."""
    ov, oe = canonical_order(vf, ee)
    perm = np.concatenate([ov, len(vf) + oe])
    h = hashlib.sha256()
    h.update(np.ascontiguousarray(hit[perm], np.uint8).tobytes())
    h.update(np.ascontiguousarray(toi[perm], np.float64).tobytes())
    return h.hexdigest()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=oracle.default_threads())
    args = ap.parse_args()
    s = scenes.perturbed_torus(seed=SEED, gadgets=GADGETS)
    t0 = time.time()
    vf, ee = oracle.broad(s.V0, s.V1, s.E, s.F, nthreads=args.threads)
    t1 = time.time()
    print(f"broad: {len(vf)} VF + {len(ee)} EE pairs in {t1 - t0:.0f} s", flush=True)
    hit, toi, n_enq, n_eval, n_axis, tmin = oracle.narrow_with_work(s.V0, s.V1, s.E, s.F, vf, ee, DELTA, MAX_ITER,
                                                                    nthreads=args.threads)
    t2 = time.time()
    print(f"narrow: {t2 - t1:.0f} s, toi_min {tmin}", flush=True)
    nvf = len(vf)
    capped = n_enq > MAX_ITER
    edges = [0, 1, 2, 10, 100, 1000, 10 ** 4, 10 ** 5, 10 ** 6, 10 ** 7]
    hist = np.histogram(n_eval, bins=edges + [np.iinfo(np.int64).max])[0]
    man = {
        "workload": f"perturbed_torus(seed={SEED}, gadgets={GADGETS})",
        "delta": DELTA, "max_iter": MAX_ITER,
        "input_sha256": scene_hash(s),
        "nv": s.nv, "ne": s.ne, "nf": s.nf,
        "n_vf": int(nvf), "n_ee": int(len(ee)),
        "pairs_sha256": pairs_hash(vf, ee),
        "results_sha256": results_hash(vf, ee, hit, toi, n_enq),
        "hit_toi_sha256": hit_toi_hash(vf, ee, hit, toi),
        "hits": int(hit.sum()),
        "toi_min": float(tmin), "toi_min_bits": int(np.float64(tmin).view(np.int64)),
        "capped_pairs": int(capped.sum()),
        "toi_min_from_capped_pair": bool(np.any(capped & (toi == tmin))),
        "toi_min_uncapped": float(toi[~capped].min()) if np.any(~capped) else float("inf"),
        "n_eval": {"vf": int(n_eval[:nvf].sum()), "ee": int(n_eval[nvf:].sum())},
        "n_axis": {"vf": int(n_axis[:nvf].sum()), "ee": int(n_axis[nvf:].sum())},
        "n_eval_capped": int(n_eval[capped].sum()),
        "n_eval_histogram": {"edges": edges, "counts": [int(c) for c in hist]},
        "oracle_seconds": {"broad": round(t1 - t0, 1), "narrow": round(t2 - t1, 1), "threads": args.threads},
        "written_by": "tests/golden/make_torus_manifest.py",
    }
    with open(OUT, "w") as f:
        json.dump(man, f, indent=1)
    print(json.dumps(man, indent=1))


if __name__ == "__main__":
    main()
