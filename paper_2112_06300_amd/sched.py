"""Learned schedule for the narrow phase: train and load the cost model.

The model (an MLP 16 -> 64 -> 64 -> 1 evaluated with bf16 weights on the
matrix cores) predicts log2(1 + intervals enqueued) of each candidate pair;
`Context.narrow(..., schedule=("learned", params, norm))` then searches pairs
in decreasing predicted cost.  Results never depend on it.

Training runs on the GPU with the library's own kernels: the plain narrow
phase logs every pair's cost (its n_enq output), ccd_features computes the
inputs, ccd_mlp_grad the gradient of the mean squared error and ccd_adam_step
the update.  PyTorch only holds the buffers, draws the minibatch indices and
computes the feature mean and deviation once.

    python -m paper_2112_06300_amd.sched --out paper_2112_06300_amd/sched_model.npz
"""
import argparse
import json
import os
import time

import numpy as np

from . import MODEL_PARAMS, NUM_FEATURES, HIDDEN, Context

HERE = os.path.dirname(os.path.abspath(__file__))
MODEL_PATH = os.path.join(HERE, "sched_model.npz")              # cloth on sphere
TORUS_MODEL_PATH = os.path.join(HERE, "sched_model_torus.npz")  # perturbed torus with degenerate gadgets
# Near-degenerate gadgets in the perturbed-torus workload: about 1 % of its candidate pairs.
TORUS_GADGETS = 12000
# Bumped whenever the feature definitions in the feature kernel change: a model
# trained on other features is refused.
FEATURE_VERSION = 1


def init_params(seed=0):
    """He-initialized float32 parameters (W1, b1, W2, b2, w3, b3)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    W1 = rng.normal(0.0, np.sqrt(2.0 / NUM_FEATURES), size=(NUM_FEATURES, HIDDEN))
    W2 = rng.normal(0.0, np.sqrt(2.0 / HIDDEN), size=(HIDDEN, HIDDEN))
    w3 = rng.normal(0.0, np.sqrt(1.0 / HIDDEN), size=HIDDEN)
    p = np.concatenate([W1.ravel(), np.zeros(HIDDEN), W2.ravel(), np.zeros(HIDDEN), w3, np.zeros(1)])
    assert p.size == MODEL_PARAMS
    return p.astype(np.float32)


def cost_logs(ctx, scene, delta=1e-6, max_iter=10 ** 6):
    """(features, labels) of every candidate pair of a scene, from the broad phase and the plain narrow
    phase (labels = log2(1 + n_enq)), both on the device."""
    import torch
    dev = lambda x, dt: torch.as_tensor(np.ascontiguousarray(x)).to("cuda", dt)
    V0, V1 = dev(scene.V0, torch.float64), dev(scene.V1, torch.float64)
    E, F = dev(scene.E, torch.int32), dev(scene.F, torch.int32)
    vf, ee = ctx.broad(V0, V1, E, F)
    _, _, _, n_enq = ctx.narrow(V0, V1, E, F, vf, ee, delta, max_iter, with_costs=True)
    feat = ctx.features(V0, V1, E, F, vf, ee, delta)
    label = torch.log2(1.0 + n_enq.to(torch.float32))
    return feat, label


def normalization(feat):
    """mean[16] then 1/std[16] of the training features (constant features get 1/std = 1)."""
    import torch
    mean = feat.mean(0)
    std = feat.std(0)
    istd = torch.where(std > 1e-6, 1.0 / std, torch.ones_like(std))
    return torch.cat([mean, istd]).to(torch.float32).contiguous()


def train(ctx, feat, label, steps=1500, batch=16384, lr=3e-3, seed=0, log_every=0, heavy_frac=0.0,
          heavy_label=10.0):
    """Adam on the mean squared error, on the GPU; returns (params, norm, history) as device tensors.

    heavy_frac: the share of every minibatch drawn from the pairs whose label is at least heavy_label (the
    few costly pairs the schedule must find among millions of cheap ones), the rest uniformly."""
    import torch
    n = feat.shape[0]
    norm = normalization(feat)
    params = torch.as_tensor(init_params(seed)).cuda()
    grad = torch.zeros(MODEL_PARAMS, dtype=torch.float32, device="cuda")
    m = torch.zeros_like(grad)
    v = torch.zeros_like(grad)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    heavy = torch.nonzero(label >= heavy_label).flatten() if heavy_frac > 0 else None
    nh = int(min(batch, n) * heavy_frac) if heavy is not None and heavy.numel() > 0 else 0
    hist = []
    for step in range(1, steps + 1):
        idx = torch.randint(0, n, (min(batch, n) - nh,), device="cuda", generator=g)
        if nh:
            idx = torch.cat([idx, heavy[torch.randint(0, heavy.numel(), (nh,), device="cuda", generator=g)]])
        fb = feat.index_select(0, idx).contiguous()
        lb = label.index_select(0, idx).contiguous()
        ctx.mlp_grad(params, norm, fb, lb, grad=grad, loss=loss)
        # cosine decay of the learning rate
        lr_t = lr * 0.5 * (1.0 + np.cos(np.pi * (step - 1) / steps))
        ctx.adam_step(params, grad, m, v, step, lr=lr_t)
        if log_every and (step % log_every == 0 or step == steps):
            hist.append((step, float(loss.item()) / fb.shape[0]))
    return params, norm, hist


def spearman(a, b):
    """Rank correlation of two 1-D arrays (average ranks for ties)."""
    from scipy.stats import spearmanr
    return float(spearmanr(np.asarray(a), np.asarray(b)).correlation)


def save_model(path, params, norm, meta):
    np.savez(path, params=np.asarray(params, np.float32), norm=np.asarray(norm, np.float32),
             feature_version=np.int64(FEATURE_VERSION), meta=np.array(json.dumps(meta)))


def load_model(path=MODEL_PATH):
    """(params, norm, meta) of a trained model as host float32 arrays; raises if it is missing or was trained
    on other features."""
    if not os.path.exists(path):
        raise FileNotFoundError(f"{path} is missing: train it with python -m paper_2112_06300_amd.sched")
    with np.load(path, allow_pickle=False) as z:
        if int(z["feature_version"]) != FEATURE_VERSION:
            raise ValueError(f"{path} was trained on feature version {int(z['feature_version'])}, "
                             f"this library computes version {FEATURE_VERSION}")
        params = z["params"].astype(np.float32)
        norm = z["norm"].astype(np.float32)
        meta = json.loads(str(z["meta"]))
    if params.size != MODEL_PARAMS or norm.size != 2 * NUM_FEATURES:
        raise ValueError(f"{path} has the wrong parameter count")
    return params, norm, meta


def main():
    ap = argparse.ArgumentParser(description="train the narrow-phase cost model on the GPU")
    ap.add_argument("--workload", choices=["cloth", "torus"], default="cloth")
    ap.add_argument("--out", default=None)
    ap.add_argument("--seeds", default=None, help="scene seeds to log costs from (cloth 12,13; torus 13)")
    ap.add_argument("--cloth-n", type=int, default=256)
    ap.add_argument("--eval-seed", type=int, default=None)
    ap.add_argument("--steps", type=int, default=1500)
    ap.add_argument("--batch", type=int, default=16384)
    ap.add_argument("--lr", type=float, default=3e-3)
    ap.add_argument("--heavy-frac", type=float, default=0.0,
                    help="share of each minibatch drawn from pairs with log2(1 + n_enq) >= --heavy-label")
    ap.add_argument("--heavy-label", type=float, default=10.0)
    ap.add_argument("--top-k", type=int, default=20000, help="report the recall of the k costliest eval pairs")
    args = ap.parse_args()
    import torch
    import scenes
    torus = args.workload == "torus"
    out = args.out or (TORUS_MODEL_PATH if torus else MODEL_PATH)
    seeds = args.seeds or ("13" if torus else "12,13")
    eval_seed = args.eval_seed if args.eval_seed is not None else (23 if torus else 22)

    def make(seed):
        if torus:
            return scenes.perturbed_torus(seed=seed, gadgets=TORUS_GADGETS)
        return scenes.cloth_on_sphere(seed=seed, n=args.cloth_n)

    ctx = Context(0)
    t0 = time.perf_counter()
    feats, labels = [], []
    for s in [int(x) for x in seeds.split(",")]:
        f, l = cost_logs(ctx, make(s))
        feats.append(f)
        labels.append(l)
        print(f"seed {s}: {f.shape[0]} pairs logged", flush=True)
    feat = torch.cat(feats).contiguous()
    label = torch.cat(labels).contiguous()
    t1 = time.perf_counter()
    params, norm, hist = train(ctx, feat, label, steps=args.steps, batch=args.batch, lr=args.lr, log_every=100,
                               heavy_frac=args.heavy_frac, heavy_label=args.heavy_label)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for step, l in hist:
        print(f"step {step}: minibatch mse {l:.4f}", flush=True)
    fe, le = cost_logs(ctx, make(eval_seed))
    pred = ctx.mlp_predict(params, norm, fe)
    rho = spearman(pred.cpu().numpy(), le.cpu().numpy())
    mse = float(((pred - le) ** 2).mean().item())
    # how many of the k costliest pairs the network ranks among its k costliest
    k = min(args.top_k, fe.shape[0])
    top_true = set(torch.topk(le, k).indices.cpu().numpy().tolist())
    top_pred = set(torch.topk(pred, k).indices.cpu().numpy().tolist())
    recall = len(top_true & top_pred) / max(1, k)
    name = f"perturbed_torus gadgets={TORUS_GADGETS}" if torus else f"cloth_on_sphere n={args.cloth_n}"
    meta = {"train": f"{name} seeds {seeds}", "pairs": int(feat.shape[0]),
            "steps": args.steps, "batch": args.batch, "lr": args.lr, "label": "log2(1 + n_enq)",
            "eval": f"{name} seed {eval_seed}", "eval_pairs": int(fe.shape[0]),
            "eval_mse": mse, "eval_spearman": rho, f"eval_top{k}_recall": recall, "heavy_frac": args.heavy_frac,
            "heavy_label": args.heavy_label, "train_seconds": t2 - t1, "log_seconds": t1 - t0}
    save_model(out, params.cpu().numpy(), norm.cpu().numpy(), meta)
    print(json.dumps(meta), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
