"""Pins of the oracle's Adam update (the optimiser of the learned indicator's
training, checked against the GPU trainer's `k_adam`).

Two facts fix it independently of its own code:
  * the closed form of the first step: from zero moments the bias-corrected
    moments are g and g^2, so every parameter moves by -lr g / (|g| + eps);
  * torch.optim.Adam (Kingma & Ba's algorithm with bias correction, the
    epsilon added to the square root of the corrected second moment) in
    float64, over several steps with changing gradients.
`check_*` take the module under test so that the mutant test can run them on
planted mistakes."""
import numpy as np
import pytest

from oracle import indicator as ind

LR, B1, B2, EPS = 3e-3, 0.9, 0.999, 1e-8


def _params(seed):
    p = ind.init_params(seed)
    rng = np.random.default_rng(seed + 100)
    p["b1"] = rng.normal(size=p["b1"].shape)   # nonzero biases too
    return p


def _grads(seed, params):
    rng = np.random.default_rng(seed)
    # magnitudes spread over decades, both signs, some exact zeros
    return {k: rng.normal(size=v.shape) * 10.0 ** rng.integers(-6, 2, size=v.shape) * (rng.uniform(size=v.shape) > 0.05)
            for k, v in params.items()}


def check_first_step_closed_form(mod):
    p = _params(1)
    p0 = {k: v.copy() for k, v in p.items()}
    g = _grads(2, p)
    mod.adam_step(p, g, {}, lr=LR, b1=B1, b2=B2, eps=EPS)
    for k in p:
        want = p0[k] - LR * g[k] / (np.abs(g[k]) + EPS)
        np.testing.assert_allclose(p[k], want, rtol=0, atol=1e-15 * (1.0 + np.abs(p0[k]).max()), err_msg=k)


def check_matches_torch(mod, steps=7):
    import torch
    p = _params(3)
    tp = {k: torch.tensor(v.copy(), dtype=torch.float64, requires_grad=True) for k, v in p.items()}
    opt = torch.optim.Adam(list(tp.values()), lr=LR, betas=(B1, B2), eps=EPS)
    state = {}
    for s in range(steps):
        g = _grads(10 + s, p)
        mod.adam_step(p, g, state, lr=LR, b1=B1, b2=B2, eps=EPS)
        opt.zero_grad()
        for k, t in tp.items():
            t.grad = torch.tensor(g[k], dtype=torch.float64)
        opt.step()
        for k in p:
            ref = tp[k].detach().numpy()
            np.testing.assert_allclose(p[k], ref, rtol=0, atol=1e-12 * (1.0 + np.abs(ref).max()),
                                       err_msg=f"step {s + 1}, {k}")


def test_first_step_is_lr_times_sign():
    check_first_step_closed_form(ind)


def test_steps_match_torch_adam():
    check_matches_torch(ind)


def test_step_count_advances_per_call():
    """The bias correction uses the number of calls so far: two calls with a
    zero gradient after one real step leave moments decaying, never reset."""
    p = _params(4)
    state = {}
    g = _grads(5, p)
    ind.adam_step(p, g, state, lr=LR)
    ind.adam_step(p, {k: np.zeros_like(v) for k, v in g.items()}, state, lr=LR)
    assert state["t"] == 2
    np.testing.assert_allclose(state["m_W1"], B1 * (1 - B1) * g["W1"], rtol=1e-15)
