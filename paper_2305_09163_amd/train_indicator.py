"""Train the learned smoothness indicator on the GPU with the library's own
kernels: harvest (stencil features, WENO5-weight labels) from FP64 runs of
the shock tube and the bubble collapse, then mean-BCE Adam steps of the bf16
matrix-core trainer.  Everything numeric runs in libmfc.so; this module only
orders the calls and draws the (seeded) sample indices.

    python -m paper_2305_09163_amd.train_indicator [--samples 1e7] [--steps N] [--out FILE]

writes the 1601 FP32 parameters (flat order of include/mfc.h) to FILE
(default: indicator_weights.npy next to this module) and, beside it, a .json
with the routing threshold chosen on held-out samples (the smallest tau
whose false-smooth rate is at most 1e-3) and the training record.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "indicator_weights.npy")
NIN, NH = 15, 32


def glorot_init(seed: int) -> np.ndarray:
    """Glorot-uniform weights and zero biases in the flat parameter order."""
    rng = np.random.default_rng(seed)
    parts = []
    for n_in, n_out in ((NIN, NH), (NH, NH), (NH, 1)):
        a = math.sqrt(6.0 / (n_in + n_out))
        parts += [rng.uniform(-a, a, size=n_in * n_out), np.zeros(n_out)]
    return np.concatenate(parts).astype(np.float32)


def harvest_runs(runs, log=print):
    """runs: list of (GridSpec, primitive state, snapshot steps, cfl).  Each run
    is advanced in FP64 by the library; every snapshot contributes all its
    interior (cell, direction) samples.  Returns device tensors (X, Y)."""
    import torch

    from . import mfc

    Xs, Ys = [], []
    for spec, w, snaps, cfl in runs:
        s = mfc.Solver(spec, kernel=mfc.MFC_KERNEL_SPLIT if spec.ndim == 3 else mfc.MFC_KERNEL_FUSED)
        q = s.state_from_prim(w)
        done = 0
        for step in snaps:
            if step > done:
                s.run(q, step - done, cfl=cfl)
                done = step
            X, Y, _ = s.harvest(q)
            Xs.append(X)
            Ys.append(Y)
        s.check()
        log(f"harvest: {spec.ndim}D {tuple(spec.n[:spec.ndim])} snapshots {list(snaps)}: "
            f"{sum(int(y.numel()) for y in Ys[-len(snaps):])} samples")
        s.close()
    return torch.cat(Xs), torch.cat(Ys)


def train(X, Y, steps: int, batch: int = 4096, lr: float = 3e-3, seed: int = 0, params=None, log=print,
          log_every: int = 500, balanced: bool = True):
    """Adam on mean BCE; batches drawn with replacement (seeded), half from
    each label when `balanced` (the classes are far from even on these
    workloads).  Returns the trained FP32 parameters and the loss history."""
    import torch

    from . import mfc

    t = mfc.Trainer(batch)
    t.set_params(glorot_init(seed) if params is None else params)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    n = int(Y.numel())
    pos = torch.nonzero(Y == 1).reshape(-1).to(torch.int32)
    neg = torch.nonzero(Y == 0).reshape(-1).to(torch.int32)
    balanced = balanced and len(pos) > 0 and len(neg) > 0
    hist = []
    for k in range(steps):
        if balanced:
            h = batch // 2
            idx = torch.cat([pos[torch.randint(0, len(pos), (h,), generator=gen, device="cuda")],
                             neg[torch.randint(0, len(neg), (batch - h,), generator=gen, device="cuda")]])
        else:
            idx = torch.randint(0, n, (batch,), generator=gen, device="cuda", dtype=torch.int32)
        t.grad(X, Y, idx)
        if k % log_every == 0 or k == steps - 1:
            _, loss = t.read_grad()
            hist.append((k, loss))
            log(f"train: step {k} loss {loss:.4f}")
        # cosine decay to 10 % of the initial rate
        t.adam(lr * (0.1 + 0.9 * 0.5 * (1.0 + math.cos(math.pi * k / max(steps - 1, 1)))))
    p = t.params()
    t.close()
    return p, hist


def evaluate(params, X, Y, tau: float = 0.5):
    """Accuracy, false-smooth rate (non-smooth samples called smooth) and the
    fraction called smooth, with the library's inference kernel."""
    from . import mfc

    t = mfc.Trainer(1)
    t.set_params(params)
    P = t.infer(X)
    t.close()
    pred = P > tau
    y = Y.bool()
    return {"accuracy": float((pred == y).float().mean()),
            "false_smooth": float((pred & ~y).float().sum() / max(int((~y).sum()), 1)),
            "called_smooth": float(pred.float().mean()),
            "labelled_smooth": float(y.float().mean())}


def choose_tau(params, X, Y, max_false_smooth: float = 1e-3):
    """The smallest threshold whose false-smooth rate (non-smooth samples
    routed to the linear stencil) on (X, Y) is at most max_false_smooth."""
    from . import mfc

    t = mfc.Trainer(1)
    t.set_params(params)
    P = t.infer(X)
    t.close()
    Pn = P[Y == 0]
    if Pn.numel() == 0:
        return 0.5
    # the (1 - max_false_smooth) quantile of the non-smooth samples' outputs
    k = int(Pn.numel() * (1.0 - max_false_smooth))
    tau = float(Pn.sort().values[min(k, Pn.numel() - 1)])
    return min(max(tau, 0.5), 0.999999)


def default_runs(n3: int = 128):
    from . import workloads as W

    tube = W.shock_tube_1d(400)
    bub = W.bubble_collapse_3d(n=n3)
    return [(tube[0], tube[1], list(range(0, 201, 10)), 0.4),
            (bub[0], bub[1], [0, 25, 50], 0.3)]


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--samples", type=float, default=1e7, help="training samples kept (drawn without replacement)")
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--n3", type=int, default=128, help="bubble grid size")
    ap.add_argument("--seed", type=int, default=230509163)
    ap.add_argument("--out", default=DEFAULT_WEIGHTS)
    args = ap.parse_args(argv)

    import torch

    torch.cuda.set_device(0)
    log = lambda m: print(m, flush=True)  # noqa: E731
    X, Y = harvest_runs(default_runs(args.n3), log)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(args.seed)
    keep = torch.randperm(int(Y.numel()), generator=gen, device="cuda")[: int(args.samples)]
    held = keep[-100000:]
    keep = keep[:-100000]
    Xt, Yt = X[keep].contiguous(), Y[keep].contiguous()
    log(f"training set: {int(Yt.numel())} samples, {float(Yt.float().mean()):.3f} labelled smooth")
    params, hist = train(Xt, Yt, args.steps, args.batch, lr=args.lr, seed=args.seed % 1000, log=log)
    Xh, Yh = X[held].contiguous(), Y[held].contiguous()
    tau = choose_tau(params, Xh, Yh)
    stats = {t: evaluate(params, Xh, Yh, t) for t in (0.5, tau)}
    for t, ev in stats.items():
        log(f"held-out, tau {t:.6f}: {ev}")
    np.save(args.out, params.astype(np.float32), allow_pickle=False)
    meta = {"tau": tau, "rule": "false-smooth rate <= 1e-3 on 100k held-out samples (floor 0.5)",
            "held_out": {str(t): ev for t, ev in stats.items()}, "samples": int(Yt.numel()),
            "labelled_smooth": float(Yt.float().mean()), "steps": args.steps, "batch": args.batch,
            "lr": args.lr, "balanced": True, "loss": hist, "bubble_n": args.n3}
    with open(os.path.splitext(args.out)[0] + ".json", "w") as f:
        json.dump(meta, f, indent=1)
    log(f"wrote {args.out} (tau {tau:.6f})")
    return 0


if __name__ == "__main__":
    sys.exit(main())
