"""Pins of the FP64 indicator reference: gradients against central finite
differences of the loss (which uses only the forward pass), the tanh GELU
against the exact erf GELU, feature normalisation properties and labels
from the oracle's WENO5 weights."""
import math

import numpy as np
import pytest

import oracle
from oracle import indicator as ind

RNG = np.random.default_rng(77)


def test_gradients_match_finite_differences():
    params = ind.init_params(3)
    X = RNG.uniform(-1, 1, size=(37, ind.NIN))
    y = (RNG.uniform(size=37) < 0.4).astype(np.float64)
    _, g = ind.loss_and_grads(params, X, y)
    h = 1e-6
    for k, W in params.items():
        flat = W.reshape(-1)
        for idx in RNG.choice(flat.size, size=min(6, flat.size), replace=False):
            old = flat[idx]
            flat[idx] = old + h
            lp, _ = ind.loss_and_grads(params, X, y)
            flat[idx] = old - h
            lm, _ = ind.loss_and_grads(params, X, y)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            an = g[k].reshape(-1)[idx]
            assert an == pytest.approx(fd, rel=1e-6, abs=1e-9), (k, idx)


def test_tanh_gelu_close_to_exact_gelu():
    x = np.linspace(-6, 6, 1001)
    exact = 0.5 * x * (1.0 + np.vectorize(math.erf)(x / math.sqrt(2.0)))
    assert np.abs(ind.gelu(x) - exact).max() < 1e-3
    assert ind.gelu(np.array([0.0]))[0] == 0.0


def test_bce_gradient_is_sigmoid_minus_label():
    """d(BCE)/dz = sigmoid(z) - y for a single sample (closed form)."""
    params = ind.init_params(1)
    params["W3"][:] = 0.0
    params["b3"][:] = 0.7
    X = RNG.uniform(-1, 1, size=(1, ind.NIN))
    for y in (0.0, 1.0):
        _, g = ind.loss_and_grads(params, X, np.array([y]))
        assert g["b3"][0] == pytest.approx(1.0 / (1.0 + math.exp(-0.7)) - y, rel=1e-12)


def test_features_are_normalised_and_scale_invariant():
    a = RNG.uniform(0, 1, size=(50, 5))
    r = RNG.uniform(1, 1000, size=(50, 5))
    p = RNG.uniform(1e4, 1e9, size=(50, 5))
    f = ind.features(a, r, p)
    assert f.shape == (50, 15)
    assert np.all(np.abs(f) <= 1.0) and np.all(f[:, [2, 7, 12]] == 0.0)
    assert np.all(np.abs(f).reshape(50, 3, 5).max(axis=2) == pytest.approx(1.0))
    f2 = ind.features(a, 3.0 * r + 5.0, 7.0 * p)   # affine changes of rho, scale of p
    np.testing.assert_allclose(f2[:, 5:], f[:, 5:], atol=1e-12)


def test_labels_from_weno_weights():
    """Smooth data gives label 1; a jump in any one variable gives 0."""
    x = 0.01 * np.arange(-2, 3)
    smooth = np.stack([1.0 + 0.1 * np.sin(x + k) for k in range(7)])
    assert ind.label(smooth) == 1
    jump = smooth.copy()
    jump[5] = np.where(np.arange(5) < 3, 1e6, 1e4)
    assert ind.label(jump) == 0


def test_adam_reduces_loss_on_separable_data():
    params = ind.init_params(5)
    X = RNG.uniform(-1, 1, size=(512, ind.NIN))
    y = (X[:, 1] + X[:, 6] > 0).astype(np.float64)
    state = {}
    l0, _ = ind.loss_and_grads(params, X, y)
    for _ in range(200):
        _, g = ind.loss_and_grads(params, X, y)
        ind.adam_step(params, g, state, lr=1e-2)
    l1, _ = ind.loss_and_grads(params, X, y)
    assert l1 < 0.5 * l0


# ------------------------------------------------------------ bf16 operands

def test_bf16_rounding_matches_torch():
    import torch
    x32 = np.concatenate([RNG.normal(size=4000) * 10.0 ** RNG.integers(-6, 6, size=4000),
                          # exact ties between two bf16 values (ties go to the even one)
                          (np.arange(1, 200) * 2 + 1) * 2.0 ** -9 + 1.0]).astype(np.float32)
    ref = torch.tensor(x32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(ind.bf16(x32.astype(np.float64)), ref)
    assert ind.bf16(np.array([1.0 + 2.0 ** -8]))[0] == 1.0            # tie -> even
    assert ind.bf16(np.array([1.0 + 3 * 2.0 ** -8]))[0] == 1.0 + 2.0 ** -6


def test_bf16_gradients_within_rounding_bound_of_fp64():
    """Rounding the product operands perturbs each by at most 2^-9 relative;
    the gradients then move by a few times that, not more."""
    params = ind.init_params(5)
    X = RNG.uniform(-1, 1, size=(512, ind.NIN))
    y = (RNG.uniform(size=512) < 0.5).astype(np.float64)
    l64, g64 = ind.loss_and_grads(params, X, y)
    l16, g16 = ind.loss_and_grads(params, X, y, bf16_operands=True)
    assert abs(l16 - l64) < 1e-2 * abs(l64)
    for k in g64:
        rel = np.linalg.norm(g16[k] - g64[k]) / np.linalg.norm(g64[k])
        assert 0 < rel < 3e-2, (k, rel)      # rounding happened, and stayed bounded


def test_flatten_round_trip_and_size():
    p = ind.init_params(1)
    f = ind.flatten(p)
    assert f.size == ind.NPARAM == 1601
    q = ind.unflatten(f)
    for k in p:
        np.testing.assert_array_equal(p[k], q[k])
    assert f[0] == p["W1"][0, 0] and f[1] == p["W1"][0, 1]        # in-major
    assert f[ind.NIN * ind.NH] == p["b1"][0]


# ------------------------------------------------------------ field harvest

def _spec2d(n=(12, 10)):
    from paper_2305_09163_amd import workloads as W
    return W.GridSpec(ndim=2, n=n)


def test_harvest_order_and_labels_on_a_y_layer():
    """A water/air layer varying only along y: every x-direction sample is
    smooth with zero deviation; y-direction samples near the layer are not."""
    from paper_2305_09163_amd import workloads as W
    spec = _spec2d()
    x, y, _ = spec.mesh()
    a1 = np.where(y < 0.5, 1 - 1e-6, 1e-6) * np.ones_like(x)
    w = W._assemble(spec, a1, 1000.0, 1.2, [0 * x, 0 * x], 1e5 * np.ones_like(x))
    q = oracle.fill_ghosts(spec, oracle.prim_to_cons_field(spec, w))
    X, Y, D = ind.harvest(spec, q)
    nc = spec.cells
    assert X.shape == (2 * nc, 15) and Y.shape == (2 * nc,)
    assert (Y[:nc] == 1).all() and (D[:nc] == 0).all() and (X[:nc] == 0).all()
    ylab = Y[nc:].reshape(spec.n[1], spec.n[0])
    assert (ylab[:, 0] == ylab[:, 5]).all()                         # rows are uniform in x
    assert ylab[3:7].min() == 0 and ylab[0].all() and ylab[-1].all()  # non-smooth only near y = 0.5
    # one sample by hand: cell (i=4, j=5), direction y
    j, i = 5, 4
    st = np.array([a1[0, j + 3 - 2 + t, i + 3] for t in range(5)])   # mesh() spans the padded grid
    np.testing.assert_allclose(X[nc + j * spec.n[0] + i, :5], ind.features(st, st, st)[:5])


# ------------------------------------------------------ routed reconstruction

def test_linear_mode_is_the_ideal_weight_limit_and_fifth_order():
    from paper_2305_09163_amd import workloads as W
    errs = []
    for n in (32, 64):
        spec, w = W.sine_advection_1d(n)
        q = oracle.prim_to_cons_field(spec, w)
        qf = oracle.fill_ghosts(spec, q)
        Llin, _ = oracle.rhs(spec, qf, oracle.RECON_LINEAR)
        import dataclasses
        big = dataclasses.replace(spec, weno_eps=1e12)
        Lbig, _ = oracle.rhs(big, qf)
        np.testing.assert_allclose(Llin, Lbig, rtol=1e-8, atol=1e-9 * np.abs(Llin).max())
        dx = spec.dx[0]
        nsteps = int(math.ceil(0.25 / min(0.4 * dx / 2.2, 2.0 * dx ** (5.0 / 3.0))))  # RK3 error below spatial
        qn, t, st = oracle.run(spec, q, nsteps, dt=0.25 / nsteps, recon=oracle.RECON_LINEAR)
        assert st == oracle.OK
        rho = qn[0, 0, 0, 3:-3] + qn[1, 0, 0, 3:-3]
        errs.append(np.abs(rho - W.sine_cell_averages(spec, t)).mean())
    # the linear stencil is fifth order from the coarsest grid on (no weights to settle)
    assert math.log2(errs[0] / errs[1]) > 4.7, errs


def test_routed_rhs_reduces_to_weno_and_linear():
    from paper_2305_09163_amd import workloads as W
    spec, w = W.droplet_shock_2d((14, 11), W.SEED + 7)
    q = oracle.fill_ghosts(spec, oracle.prim_to_cons_field(spec, w))
    params = ind.init_params(2)
    Lw, _ = oracle.rhs(spec, q)
    Ll, _ = oracle.rhs(spec, q, oracle.RECON_LINEAR)
    L0, _, P = ind.rhs_learned(spec, q, params, tau=2.0)    # P < 2: never linear
    L1, _, _ = ind.rhs_learned(spec, q, params, tau=-1.0)   # P > -1: always linear
    np.testing.assert_array_equal(L0, Lw)
    np.testing.assert_array_equal(L1, Ll)
    # P exists exactly on reconstruction cells: -1 .. n along d, interior across
    ok = ~np.isnan(P)
    assert ok[0].sum() == (spec.n[0] + 2) * spec.n[1] and ok[1].sum() == spec.n[0] * (spec.n[1] + 2)
    # a mask that selects linear only in the x direction: y-faces unchanged
    mask = np.zeros_like(P, dtype=np.uint8)
    mask[0] = 1
    Lx, _ = oracle.rhs(spec, q, oracle.RECON_MASK, mask)
    assert not np.array_equal(Lx, Lw) and not np.array_equal(Lx, Ll)


def test_learned_run_with_no_routing_is_the_oracle_run():
    from paper_2305_09163_amd import workloads as W
    spec, w = W.shock_tube_1d(60)
    q = oracle.prim_to_cons_field(spec, w)
    a, ta, sa = oracle.run(spec, q, 3, cfl=0.4)
    b, tb, sb, frac = ind.run_learned(spec, q, ind.init_params(0), 2.0, 3, 0.4)
    assert sa == sb == oracle.OK and frac == 0.0 and ta == tb
    np.testing.assert_array_equal(a[:, :, :, 3:-3], b[:, :, :, 3:-3])
