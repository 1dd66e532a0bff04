"""Writes indicator_oracle_trained.npy: the learned-indicator network trained
by the FP64 reference alone (oracle.indicator: harvest, forward/backward,
Adam), used by the GPU tests as a network that does separate smooth from
non-smooth stencils, so that routing by it keeps WENO5 at interfaces.

    python tests/golden/make_indicator_params.py
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from oracle import indicator as ind  # noqa: E402
from paper_2305_09163_amd import workloads as W  # noqa: E402

OUT = os.path.join(HERE, "indicator_oracle_trained.npy")


def samples():
    runs = [(W.shock_tube_1d(400), [0, 20, 40], 0.4),
            (W.droplet_shock_2d(40, W.SEED + 11), [0, 2], 0.3),
            (W.bubble_collapse_3d(n=20), [0, 3], 0.3),
            (W.sine_advection_1d(64), [0], 0.4)]
    X, Y = [], []
    for (spec, w), snaps, cfl in runs:
        q = oracle.prim_to_cons_field(spec, w)
        done = 0
        for s in snaps:
            if s > done:
                q, _, st = oracle.run(spec, q, s - done, cfl=cfl)
                assert st == oracle.OK
                done = s
            x, y, _ = ind.harvest(spec, oracle.fill_ghosts(spec, q))
            X.append(x)
            Y.append(y)
    return np.concatenate(X), np.concatenate(Y).astype(np.float64)


def main():
    X, Y = samples()
    rng = np.random.default_rng(20230516)
    params = ind.init_params(0)
    state = {}
    for step in range(600):
        idx = rng.integers(0, len(Y), size=2048)
        loss, g = ind.loss_and_grads(params, X[idx], Y[idx])
        ind.adam_step(params, g, state, lr=3e-3)
        if step % 100 == 0:
            print(f"step {step} loss {loss:.4f}", flush=True)
    P, _ = ind.forward(params, X)
    print(f"{len(Y)} samples, {Y.mean():.3f} smooth; accuracy {((P > 0.5) == (Y > 0.5)).mean():.3f}")
    np.save(OUT, ind.flatten(params).astype(np.float32), allow_pickle=False)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
