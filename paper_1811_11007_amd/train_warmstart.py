"""Train the NNI warm-start network on lengths the optimiser itself produces.

  python -m paper_1811_11007_amd.train_warmstart --out <weights.json>

1. Simulates 64 taxa x 2500 sites under GTR+G4 (exchangeabilities
   ~ Dirichlet(1 x 6), frequencies ~ Dirichlet(10 x 4), alpha 0.5) on a Yule
   tree with Exp(mean 0.05) lengths, seed 5.
2. Fully optimises the generating topology (the start tree) and runs the
   threshold search from it, optimising for each proposal every length
   (--target full, the default and the shipped weights) or only its five
   touched lengths with the rest held at the parent's (--target touched),
   and recording for each proposed neighbour
   the features of its move in the parent and its five optimised touched
   lengths beside the parent's.  The targets are
   log((t_new + s) / (t_parent + s)) with s = 1e-4, so lengths at or near
   the lower bound do not dominate the loss.
   The collection threshold widens until the sample target is reached.
3. Trains the 14 -> 128 (tanh) -> 5 perceptron on the GPU with the
   library's own forward, backward and Adam kernels (minibatches, mean
   squared error), folds the feature standardisation into the first layer,
   and writes the parameters with the training record as JSON.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def workload(seed, n=64, sites=2500):
    import synth
    rng = np.random.default_rng(seed)
    e, b = synth.yule_tree(n, rng, mean=0.05)
    aln = synth.make_alignment(e, b, n, sites, rng, alpha=0.5, n_cats=4)
    return e, b, aln


def optimise_start(ctx, A, e, b):
    import torch
    from . import _lib as L
    dev = torch.device("cuda", 0)
    plan = L.Plan(ctx, [A], L.Trees([e]), L.PT_PLAN_OPTIMIZE, L.PT_FP32)
    B = torch.tensor(b, dtype=torch.float64, device=dev)
    lnl = torch.zeros(1, dtype=torch.float64, device=dev)
    plan.optimize(B, lnl)
    torch.cuda.synchronize()
    out = B.cpu().numpy(), float(lnl.item())
    plan.close()
    return out


def train(ctx, X, Y, n_hidden=128, epochs=40, batch=4096, lr=2e-3, seed=0, val_frac=0.1):
    """Trains on the GPU; returns (params with the standardisation folded in, record)."""
    import torch
    from . import _lib as L
    dev = torch.device("cuda", 0)
    rng = np.random.default_rng(seed)
    idx = rng.permutation(len(X))
    n_val = max(1, int(len(X) * val_frac))
    va, tr = idx[:n_val], idx[n_val:]
    mu = X[tr].mean(axis=0)
    sd = X[tr].std(axis=0) + 1e-6
    Xs = ((X - mu) / sd).astype(np.float32)
    ni, no = X.shape[1], Y.shape[1]
    W1 = rng.normal(0, np.sqrt(1.0 / ni), (ni, n_hidden))
    W2 = rng.normal(0, np.sqrt(1.0 / n_hidden), (n_hidden, no)) * 0.1
    p0 = np.concatenate([W1.ravel(), np.zeros(n_hidden), W2.ravel(), np.zeros(no)]).astype(np.float32)
    net = L.MLP(ctx, ni, n_hidden, no, p0)
    Xt = torch.tensor(Xs[tr], device=dev)
    Yt = torch.tensor(Y[tr], device=dev)
    Xv = torch.tensor(Xs[va], device=dev)
    Yv = torch.tensor(Y[va], device=dev)
    loss = torch.zeros(1, dtype=torch.float64, device=dev)
    g = torch.empty(net.n_params, dtype=torch.float32, device=dev)

    def mse(Xd, Yd):
        net.gradient(Xd, Yd, g, loss)
        return loss.item() / Yd.numel()

    hist = []
    steps = 0
    t0 = time.perf_counter()
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    for ep in range(epochs):
        lr_ep = lr * (0.5 * (1 + np.cos(np.pi * ep / epochs)))
        perm = torch.randperm(len(tr), device=dev, generator=gen)
        for s in range(0, len(tr), batch):
            sel = perm[s:s + batch]
            net.train_step(Xt[sel].contiguous(), Yt[sel].contiguous(), lr=float(lr_ep))
            steps += 1
        if ep % 5 == 4 or ep == epochs - 1:
            hist.append((ep + 1, mse(Xt, Yt), mse(Xv, Yv)))
            log("epoch %d train %.5f val %.5f" % hist[-1])
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    p = net.params().astype(np.float64)
    net.close()
    # fold x_std = (x - mu) / sd into the first layer
    W1 = p[:ni * n_hidden].reshape(ni, n_hidden)
    b1 = p[ni * n_hidden:ni * n_hidden + n_hidden]
    W1f = W1 / sd[:, None]
    b1f = b1 - (mu / sd) @ W1
    pf = p.copy()
    pf[:ni * n_hidden] = W1f.ravel()
    pf[ni * n_hidden:ni * n_hidden + n_hidden] = b1f
    rec = {"train_rows": int(len(tr)), "val_rows": int(n_val), "epochs": epochs, "batch": batch, "lr": lr,
           "adam_steps": steps, "train_seconds": round(secs, 2),
           "history": [{"epoch": e, "train_mse": round(a, 6), "val_mse": round(b, 6)} for e, a, b in hist],
           "val_mse_zero_prediction": round(float(np.mean(Y[va] ** 2)), 6)}
    return pf.astype(np.float32), rec


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--seed", type=int, default=5)
    ap.add_argument("--samples", type=int, default=100000)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--shift", type=float, default=1e-4)
    ap.add_argument("--target", choices=["full", "touched"], default="full",
                    help="full: every length optimised (the shipped weights); touched: only the five touched "
                         "lengths, the rest held at the parent's")
    ap.add_argument("--save-data", default=None, help="also write the collected samples (.npz)")
    args = ap.parse_args()
    import torch  # noqa: F401
    from . import _lib as L
    from .search import ThresholdSearch

    ctx = L.Context(0)
    e, b, aln = workload(args.seed)
    A = L.Alignment.from_synth(ctx, aln)
    b0, l0 = optimise_start(ctx, A, e, b)
    log("start tree lnL %.4f, %d patterns" % (l0, aln.n_patterns))
    samples = []
    colls = []
    for T in (-10.0, -30.0, -100.0, -300.0, -1000.0):
        t0 = time.perf_counter()
        res = ThresholdSearch(ctx, A, threshold=T, batch=1024).run(
            [(e, b0)], collect=args.target, max_samples=args.samples, progress=log)
        samples = res.samples
        colls.append({"threshold": T, "samples": len(samples), "good": len(res.good), "visited": res.visited,
                      "seconds": round(time.perf_counter() - t0, 2)})
        log("collect T=%g: %d samples, %d good, %d visited" % (T, len(samples), len(res.good), res.visited))
        if len(samples) >= args.samples:
            break
    X = np.stack([s[0] for s in samples]).astype(np.float64)
    Tp = np.stack([s[1] for s in samples])
    Tn = np.stack([s[2] for s in samples])
    if args.save_data:
        np.savez_compressed(args.save_data, X=X.astype(np.float32), t_parent=Tp, t_new=Tn)
    Y = (np.log(Tn + args.shift) - np.log(np.maximum(Tp, 0.0) + args.shift)).astype(np.float32)
    params, rec = train(ctx, X, Y, epochs=args.epochs)
    out = {"n_in": L.PT_NNI_FEATURES, "n_hidden": 128, "n_out": 5, "shift": args.shift,
           "workload": "64 taxa x 2500 sites GTR+G4 (seed %d, %d patterns)" % (args.seed, aln.n_patterns),
           "target": args.target, "collection": colls, "samples": len(samples), "training": rec,
           "params": [float(x) for x in params]}
    json.dump(out, open(args.out, "w"))
    log("wrote", args.out)
    ctx.close()


if __name__ == "__main__":
    main()
