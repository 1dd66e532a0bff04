"""Learned smoothness indicator on the GPU against the oracle's reference
(oracle/indicator.py): harvested features and labels, network inference,
gradients and Adam steps of the bf16 matrix-core trainer, and the routed
right-hand side (reduction to WENO5 and to the linear scheme, and routing by
a network with decisions compared against the oracle's, taken at the same
bf16 rounding points)."""
import sys

import numpy as np
import pytest
import torch

import oracle
from oracle import indicator as ind
from parity_util import rel_linf, rhs_err
from paper_2305_09163_amd import mfc
from paper_2305_09163_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def bits_to_float(b):
    """bf16 bit patterns (int16 array) -> float64."""
    u = np.asarray(b).astype(np.uint16).astype(np.uint32) << 16
    return u.view(np.float32).astype(np.float64)


def float_to_bits(x):
    """Values already representable in bf16 -> int16 bit patterns."""
    f = np.asarray(x, dtype=np.float32)
    return (f.view(np.uint32) >> 16).astype(np.uint16).view(np.int16)


def oracle_state(spec, w, steps=0, cfl=0.3):
    q = oracle.prim_to_cons_field(spec, w)
    if steps:
        q, _, st = oracle.run(spec, q, steps, cfl=cfl)
        assert st == oracle.OK
    return oracle.fill_ghosts(spec, q)


HARVEST = {
    "bubble_3d_20x18x16": (lambda: W.bubble_collapse_3d(n=(20, 18, 16)), 3),
    "droplet_2d_40": (lambda: W.droplet_shock_2d(40, W.SEED + 11), 3),
    "shock_tube_400": (lambda: W.shock_tube_1d(400), 40),
}


def params32(seed, w3_scale=1.0, bias=0.0):
    """Oracle initial parameters (optionally with W3 scaled and random biases
    of standard deviation `bias`) rounded to FP32, the trainer's master format."""
    p = ind.init_params(seed)
    p["W3"] = p["W3"] * w3_scale
    if bias:
        rng = np.random.default_rng(seed + 1000)
        for k in ("b1", "b2", "b3"):
            p[k] = rng.normal(0.0, bias, size=p[k].shape)
    return ind.unflatten(ind.flatten(p).astype(np.float32).astype(np.float64))


@pytest.mark.parametrize("name", sorted(HARVEST))
def test_harvest_matches_oracle(name):
    make, steps = HARVEST[name]
    spec, w = make()
    say(f"[harvest] {name}")
    q = oracle_state(spec, w, steps)
    Xo, Yo, Do = ind.harvest(spec, q)
    s = mfc.Solver(spec)
    X, Y, D = s.harvest(torch.tensor(q).cuda())
    X, Y, D = X.cpu().numpy(), Y.cpu().numpy(), D.cpu().numpy()
    assert X.shape == (spec.ndim * spec.cells, 16) and (X[:, 15] == 0).all()
    # deviations: the same definition in FP64, but the weights of nearly
    # equal smoothness indicators (smooth data, where beta_r differ by
    # O(curvature) against O(slope^2)) amplify the rounding differences of
    # the two sides' primitive recovery and sums; the labels must agree
    # wherever the oracle's deviation is not within 1e-3 of the 0.01 threshold
    dd = np.abs(D - Do)
    say(f"    deviation: max |diff| {dd.max():.2e}, share above 1e-9 {(dd > 1e-9).mean():.3f}, "
        f"median {np.median(dd):.1e}")
    assert dd.max() < 2e-4 and np.median(dd) < 1e-10
    clear = np.abs(Do - 0.01) > 1e-3
    assert (Y[clear] == Yo[clear]).all()
    say(f"    samples {len(Y)}, smooth {Yo.mean():.3f}, labels within 1e-3 of the threshold: {(~clear).sum()}, "
        f"of which differ: {(Y[~clear] != Yo[~clear]).sum()}")
    # features: alpha1 and rho stencils are copies of the state on both sides,
    # so their features agree bit for bit; pressure comes from each side's own
    # recovery, and in uniform regions (differences at rounding level, scaled
    # by sqrt(eps)) its features are rounding noise
    F = bits_to_float(X[:, :15])
    Fo = ind.bf16(Xo)
    np.testing.assert_array_equal(F[:, :10], Fo[:, :10])
    # rounding noise of a pressure difference: a few hundred ulps of p (the
    # recovery subtracts Pi ~ 8e8 Pa in water), over the sqrt(eps) floor
    wq, _ = oracle.cons_to_prim_field(spec, q)
    p_cell = np.abs(wq[spec.nvar - 2][spec.interior[1:]]).reshape(-1)
    noise = 512 * np.finfo(np.float64).eps * np.tile(p_cell, spec.ndim) / np.sqrt(spec.weno_eps)
    bad = np.abs(F[:, 10:] - Fo[:, 10:]) > 2.0 ** -7 * np.abs(Fo[:, 10:]) + noise[:, None] + 1e-12
    assert not bad.any(), (bad.sum(), np.argwhere(bad)[:5])
    say(f"    pressure features bitwise equal: {(F[:, 10:] == Fo[:, 10:]).mean():.3f}")


def test_inference_matches_oracle():
    spec, w = W.bubble_collapse_3d(n=(20, 18, 16))
    Xo, _, _ = ind.harvest(spec, oracle_state(spec, w, 3))
    Xb = ind.bf16(Xo)
    params = params32(4, w3_scale=4.0)
    Po, _ = ind.forward(params, Xb, bf16_operands=True)
    t = mfc.Trainer(1 << 16)
    t.set_params(ind.flatten(params))
    Xd = torch.tensor(np.concatenate([float_to_bits(Xb), np.zeros((len(Xb), 1), np.int16)], axis=1)).cuda()
    P = t.infer(Xd).cpu().numpy().astype(np.float64)
    d = np.abs(P - Po)
    say(f"[infer] {len(P)} samples: max |dP| {d.max():.2e}, median {np.median(d):.2e}")
    assert np.median(d) < 1e-6 and d.max() < 2e-3


def _grad_case(n=3000, seed=6):
    spec, w = W.bubble_collapse_3d(n=(20, 18, 16))
    Xo, Yo, _ = ind.harvest(spec, oracle_state(spec, w, 3))
    rng = np.random.default_rng(seed)
    idx = rng.choice(len(Yo), size=n, replace=False).astype(np.int32)
    Xb = ind.bf16(Xo)
    Xd = torch.tensor(np.concatenate([float_to_bits(Xb), np.zeros((len(Xb), 1), np.int16)], axis=1)).cuda()
    Yd = torch.tensor(Yo).cuda()
    return Xb, Yo, Xd, Yd, idx


def test_gradients_match_oracle():
    Xb, Yo, Xd, Yd, idx = _grad_case()
    params = params32(7)
    t = mfc.Trainer(4096)
    t.set_params(ind.flatten(params))
    t.grad(Xd, Yd, torch.tensor(idx).cuda())
    g, loss = t.read_grad()
    lo, go = ind.loss_and_grads(params, Xb[idx], Yo[idx].astype(np.float64), bf16_operands=True)
    l64, g64 = ind.loss_and_grads(params, Xb[idx], Yo[idx].astype(np.float64))
    gd = ind.unflatten(g.astype(np.float64))
    say(f"[grad] loss gpu {loss:.7f} oracle {lo:.7f}")
    assert abs(loss - lo) < 1e-5 * abs(lo)
    for k in go:
        rel = np.linalg.norm(gd[k] - go[k]) / np.linalg.norm(go[k])
        rel64 = np.linalg.norm(gd[k] - g64[k]) / np.linalg.norm(g64[k])
        say(f"    {k}: rel err vs bf16-operand oracle {rel:.2e}, vs FP64 oracle {rel64:.2e}")
        assert rel < 2e-3, k
        assert rel64 < 3e-2, k
    # deterministic: the same call gives the same bits
    t.grad(Xd, Yd, torch.tensor(idx).cuda())
    g2, _ = t.read_grad()
    assert np.array_equal(g, g2)


def test_adam_steps_match_oracle():
    Xb, Yo, Xd, Yd, idx = _grad_case(2048, seed=8)
    params = params32(9)
    t = mfc.Trainer(2048)
    t.set_params(ind.flatten(params))
    ref = {k: v.copy() for k, v in params.items()}
    state = {}
    lr = 1e-3
    for step in range(3):
        t.grad(Xd, Yd, torch.tensor(idx).cuda())
        t.adam(lr)
        _, go = ind.loss_and_grads(ref, Xb[idx], Yo[idx].astype(np.float64), bf16_operands=True)
        ind.adam_step(ref, go, state, lr=lr)
    got = ind.unflatten(t.params().astype(np.float64))
    for k in ref:
        d = np.abs(got[k] - ref[k]) / lr
        # each Adam step moves a weight by about lr; gradients that differ by
        # rounding give steps that differ by far less than lr
        say(f"[adam] {k}: max |w_gpu - w_oracle| / lr = {d.max():.3e}")
        assert np.median(d) < 1e-2 and d.max() < 0.5, k


def test_training_reduces_loss():
    spec, w = W.bubble_collapse_3d(n=24)
    s = mfc.Solver(spec)
    q = s.state_from_prim(w)
    Xs, Ys = [], []
    for _ in range(3):
        X, Y, _ = s.harvest(q)
        Xs.append(X)
        Ys.append(Y)
        s.run(q, 4, cfl=0.3)
    X, Y = torch.cat(Xs), torch.cat(Ys)
    rng = np.random.default_rng(10)
    t = mfc.Trainer(4096)
    t.set_params(ind.flatten(params32(11)).astype(np.float32))
    losses = []
    for step in range(300):
        idx = torch.tensor(rng.integers(0, len(Y), size=4096).astype(np.int32)).cuda()
        t.grad(X, Y, idx)
        if step % 50 == 0 or step == 299:
            losses.append(t.read_grad()[1])
        t.adam(3e-3)
    P = t.infer(X).cpu().numpy()
    acc = ((P > 0.5) == (Y.cpu().numpy() == 1)).mean()
    say(f"[train] losses {np.round(losses, 4)}, accuracy {acc:.3f}, smooth fraction {Y.float().mean().item():.3f}")
    assert losses[-1] < 0.7 * losses[0]
    assert acc > 0.85


# -------------------------------------------------------- routed right-hand side

ROUTED = {
    "shock_tube_400": (lambda: W.shock_tube_1d(400), 30, ["fused"]),
    "droplet_2d_37x29": (lambda: W.droplet_shock_2d((37, 29), W.SEED + 12), 2, ["fused"]),
    "bubble_3d_37x21x19": (lambda: W.bubble_collapse_3d(n=(37, 21, 19)), 2, ["fused", "split"]),
}
# The linear stencil everywhere is only physical on smooth states: across a
# water/air interface its overshoots give negative mixture pressures.
LINEAR = {
    "sine_1d_64": (lambda: W.sine_advection_1d(64), 0, ["fused"]),
    "droplet_2d_37x29": (lambda: W.droplet_shock_2d((37, 29), W.SEED + 12), 2, ["fused"]),
    "smooth_3d_18": (lambda: W.random_smooth_periodic(3, 18), 0, ["fused", "split"]),
}
KERNELS = {"fused": mfc.MFC_KERNEL_FUSED, "split": mfc.MFC_KERNEL_SPLIT}
CASES = [(n, k) for n, (_, _, ks) in ROUTED.items() for k in ks]
LIN_CASES = [(n, k) for n, (_, _, ks) in LINEAR.items() for k in ks]


def gpu_rhs(spec, q, kernel, precision=mfc.MFC_FP64, params=None, tau=None):
    recon = mfc.MFC_RECON_WENO5 if params is None else mfc.MFC_RECON_LEARNED
    s = mfc.Solver(spec, precision=precision, recon=recon, kernel=KERNELS[kernel])
    if params is not None:
        s.set_indicator(ind.flatten(params), tau)
    qd = torch.tensor(q, dtype=s.dtype).cuda()
    s.fill_ghosts(qd)
    out = s.rhs(qd)
    s.check()
    return out.cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("name,kernel", CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_routing_nothing_is_weno(name, kernel, prec):
    make, steps, _ = ROUTED[name]
    spec, w = make()
    say(f"[route none] {name} {kernel} {prec}")
    q = oracle_state(spec, w, steps)
    P = {"fp64": mfc.MFC_FP64, "fp32": mfc.MFC_FP32_MIXED}[prec]
    a = gpu_rhs(spec, q, kernel, P)
    b = gpu_rhs(spec, q, kernel, P, params32(1), tau=2.0)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("name,kernel", LIN_CASES)
def test_routing_everything_is_the_linear_scheme(name, kernel):
    make, steps, _ = LINEAR[name]
    spec, w = make()
    say(f"[route all] {name} {kernel}")
    q = oracle_state(spec, w, steps)
    got = gpu_rhs(spec, q, kernel, params=params32(1), tau=-1.0)
    ref, st = oracle.rhs(spec, q, oracle.RECON_LINEAR)
    assert st == oracle.OK
    err = rhs_err(got, ref, q, spec)
    say(f"    rhs err {err.max():.2e}")
    assert err.max() <= 1e-12, err


def tau_candidates(P, margin, lo=0.05, hi=0.95):
    """Thresholds that route between lo and hi of the reconstructions to the
    linear stencil, fewest oracle outputs within `margin` first (identical
    stencils give identical outputs, so outputs cluster)."""
    Ps = np.sort(P)
    cand = np.linspace(Ps[0], Ps[-1], 2001)
    frac = 1.0 - np.searchsorted(Ps, cand, side="right") / len(Ps)
    near = np.searchsorted(Ps, cand + margin) - np.searchsorted(Ps, cand - margin)
    ok = (frac > lo) & (frac < hi)
    order = np.argsort(near[ok], kind="stable")
    return [float(c) for c in cand[ok][order]]


def ambiguous_cells(spec, P, tau, margin):
    """Interior cells whose right-hand side depends on a reconstruction whose
    oracle output lies within `margin` of tau (the two sides may route it
    differently at bf16/FP32 rounding): a reconstruction at cell c along d
    feeds the faces of c, so the cells c-1, c, c+1 along d."""
    amb = np.nan_to_num(np.abs(P - tau), nan=np.inf) < margin      # [ndim, *padded]
    bad = np.zeros(spec.shape[1:], dtype=bool)
    axis = {0: 2, 1: 1, 2: 0}
    for d in range(spec.ndim):
        a = amb[d]
        bad |= a | np.roll(a, 1, axis=axis[d]) | np.roll(a, -1, axis=axis[d])
    return bad[spec.interior[1:]]


def masked_rhs_err(got, ref, q, spec, skip):
    keep = ~skip
    g = got.copy()
    g[(slice(None),) + spec.interior[1:]] = np.where(keep, got[(slice(None),) + spec.interior[1:]],
                                                     ref[(slice(None),) + spec.interior[1:]])
    return rhs_err(g, ref, q, spec)


GOLDEN_NET = __import__("os").path.join(__import__("os").path.dirname(__file__), "golden",
                                        "indicator_oracle_trained.npy")


def golden_params():
    """A network trained by the FP64 reference alone (tests/golden/make_indicator_params.py)."""
    return ind.unflatten(np.load(GOLDEN_NET, allow_pickle=False).astype(np.float64))


@pytest.mark.parametrize("name,kernel", CASES)
def test_routed_rhs_matches_oracle(name, kernel):
    """The oracle-trained network, tau where between 2 % and 95 % of the
    reconstructions are routed to the linear stencil.  Both sides decide at
    the same bf16 rounding points; outputs within 2e-3 of tau may still be
    decided differently (FP32 against FP64 sums), so the cells they feed are
    left out of the comparison, and everything else must agree."""
    make, steps, _ = ROUTED[name]
    spec, w = make()
    q = oracle_state(spec, w, steps)
    params = golden_params()
    P = ind.smooth_probability(spec, q, params)
    Pv = P[~np.isnan(P)]
    # a threshold whose routing the oracle evaluates without non-physical
    # face states
    for tau in tau_candidates(Pv, 2e-3, lo=0.02)[:40:4]:
        ref, st, _ = ind.rhs_learned(spec, q, params, tau)
        if st == oracle.OK:
            break
    assert st == oracle.OK
    skip = ambiguous_cells(spec, P, tau, 2e-3)
    frac = (Pv > tau).mean()
    say(f"[route net] {name} {kernel}: tau {tau:.4f}, routed to linear {frac:.3f}, "
        f"cells left out {skip.mean():.4f}")
    assert 0.02 < frac < 0.95 and skip.mean() < 0.2
    got = gpu_rhs(spec, q, kernel, params=params, tau=tau)
    err = masked_rhs_err(got, ref, q, spec, skip)
    say(f"    rhs err {err.max():.2e}")
    assert err.max() <= 1e-12, err


def test_routed_linear_step_matches_oracle():
    """One SSP-RK3 step with every reconstruction routed to the linear
    stencil, against the oracle's linear scheme."""
    spec, w = W.droplet_shock_2d((37, 29), W.SEED + 12)
    q0 = oracle.prim_to_cons_field(spec, w)
    qo, t, st = oracle.run(spec, q0, 1, cfl=0.3, recon=oracle.RECON_LINEAR)
    assert st == oracle.OK
    s = mfc.Solver(spec, recon=mfc.MFC_RECON_LEARNED)
    s.set_indicator(ind.flatten(params32(3)), -1.0)
    qd = torch.tensor(q0).cuda()
    s.step(qd, cfl=0.3)
    s.check()
    err = rel_linf(qd.cpu().numpy(), qo, spec)
    say(f"[route step] rel Linf {err.max():.2e}")
    assert err.max() <= 1e-12, err


# Characteristic faces (Sec. 3.3) with the routed reconstruction: the split
# kernels keep the normal terms of their own (routed) reconstruction for the
# boundary pass, so routing and boundary treatment compose as in the oracle.
ALL_CHAR = (2, 2, 2, 2, 2, 2)


def _characteristic(sw):
    import dataclasses
    spec, w = sw
    return dataclasses.replace(spec, bc=ALL_CHAR), w


CHAR_ROUTED = {
    "bubble_3d_37x21x19": (lambda: _characteristic(W.bubble_collapse_3d(n=(37, 21, 19))), 2),
    "smooth_3d_18": (lambda: _characteristic(W.random_smooth_periodic(3, 18)), 0),
}


@pytest.mark.parametrize("name", sorted(CHAR_ROUTED))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_characteristic_routing_nothing_is_weno(name, prec):
    make, steps = CHAR_ROUTED[name]
    spec, w = make()
    say(f"[route none, characteristic faces] {name} {prec}")
    q = oracle_state(spec, w, steps)
    P = {"fp64": mfc.MFC_FP64, "fp32": mfc.MFC_FP32_MIXED}[prec]
    a = gpu_rhs(spec, q, "split", P)
    b = gpu_rhs(spec, q, "split", P, params32(1), tau=2.0)
    assert np.array_equal(a, b)


def test_characteristic_routing_everything_is_the_linear_scheme():
    spec, w = CHAR_ROUTED["smooth_3d_18"][0]()
    q = oracle_state(spec, w)
    got = gpu_rhs(spec, q, "split", params=params32(1), tau=-1.0)
    ref, st = oracle.rhs(spec, q, oracle.RECON_LINEAR)
    assert st == oracle.OK
    err = rhs_err(got, ref, q, spec)
    say(f"[route all, characteristic faces] rhs err {err.max():.2e}")
    assert err.max() <= 1e-12, err


def test_characteristic_routed_rhs_matches_oracle():
    """As test_routed_rhs_matches_oracle, with every face characteristic."""
    make, steps = CHAR_ROUTED["bubble_3d_37x21x19"]
    spec, w = make()
    q = oracle_state(spec, w, steps)
    params = golden_params()
    P = ind.smooth_probability(spec, q, params)
    Pv = P[~np.isnan(P)]
    for tau in tau_candidates(Pv, 2e-3, lo=0.02)[:40:4]:
        ref, st, _ = ind.rhs_learned(spec, q, params, tau)
        if st == oracle.OK:
            break
    assert st == oracle.OK
    skip = ambiguous_cells(spec, P, tau, 2e-3)
    frac = (Pv > tau).mean()
    say(f"[route net, characteristic faces] tau {tau:.4f}, routed to linear {frac:.3f}, "
        f"cells left out {skip.mean():.4f}")
    assert 0.02 < frac < 0.95 and skip.mean() < 0.2
    got = gpu_rhs(spec, q, "split", params=params, tau=tau)
    err = masked_rhs_err(got, ref, q, spec, skip)
    say(f"    rhs err {err.max():.2e}")
    assert err.max() <= 1e-12, err

