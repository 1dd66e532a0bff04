"""Pins of the oracle on non-uniform (tanh-stretched) cells (Sec. 4.1 grid
stretching; the WENO5 of Sec. 3.2 with cell widths Delta x_i), each against
what fixes it independently of the implementation:

  * the candidate polynomials reproduce the cell averages of any quadratic
    exactly, and with the ideal weights (epsilon -> infinity) the
    reconstruction is exact for any quartic (fifth order), both checked by
    exact integration over the non-uniform cells;
  * the smoothness indicator of a quadratic's stencil is the Jiang-Shu
    integral sum_l h^{2l-1} int (p^(l))^2 evaluated in closed form;
  * on uniform faces it is the uniform-grid WENO5 (up to rounding);
  * mirrored widths and mirrored data give mirrored face values;
  * the advected sine on a stretched periodic grid converges at fifth order;
  * partial masses, momentum and energy are conserved to round-off on a
    stretched periodic box (flux differences with per-cell widths);
  * the CFL step is cfl times the smallest Delta x / (|u| + c).
"""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from paper_2305_09163_amd import workloads as W


def poly_avg(c, a, b):
    """Average over [a, b] of sum_k c[k] x^k."""
    return sum(ck * (b ** (k + 1) - a ** (k + 1)) / (k + 1) for k, ck in enumerate(c)) / (b - a)


def weno5_face(widths, avgs, eps):
    """Face values of the middle cell of five cells with these widths."""
    return oracle.weno5_nonuniform(np.asarray(widths, float), np.asarray(avgs, float), eps)


@pytest.mark.parametrize("seed", range(20))
def test_quadratics_exact_and_quartics_exact_with_ideal_weights(seed):
    rng = np.random.default_rng(W.SEED + 60 + seed)
    widths = rng.uniform(0.5, 2.0, size=5)
    f = np.concatenate([[0.0], np.cumsum(widths)])
    for deg, eps in ((2, 1e-6), (4, 1e30)):
        c = rng.normal(size=deg + 1)
        avgs = [poly_avg(c, f[t], f[t + 1]) for t in range(5)]
        plus, minus = weno5_face(widths, avgs, eps)
        exact = lambda x: sum(ck * x ** k for k, ck in enumerate(c))  # noqa: E731
        scale = 1 + np.abs(avgs).max()
        assert plus == pytest.approx(exact(f[3]), abs=1e-11 * scale), (deg, widths)
        assert minus == pytest.approx(exact(f[2]), abs=1e-11 * scale), (deg, widths)


def test_uniform_widths_give_the_uniform_weno5():
    rng = np.random.default_rng(W.SEED + 61)
    for _ in range(50):
        s = rng.normal(size=5) * 10 ** rng.uniform(-3, 3)
        h = 10 ** rng.uniform(-3, 0)
        a = weno5_face(np.full(5, h), s, 1e-6)
        b = oracle.weno5(s, 1e-6)[:2]
        scale = np.abs(s).max()
        assert a[0] == pytest.approx(b[0], abs=1e-12 * scale) and a[1] == pytest.approx(b[1], abs=1e-12 * scale)


def test_mirror_symmetry():
    rng = np.random.default_rng(W.SEED + 62)
    for _ in range(50):
        widths = rng.uniform(0.3, 3.0, size=5)
        s = rng.normal(size=5)
        plus, minus = weno5_face(widths, s, 1e-6)
        plus_r, minus_r = weno5_face(widths[::-1].copy(), s[::-1].copy(), 1e-6)
        assert plus == pytest.approx(minus_r, rel=1e-12, abs=1e-13)
        assert minus == pytest.approx(plus_r, rel=1e-12, abs=1e-13)


def test_smoothness_indicator_is_the_jiang_shu_integral():
    """For data from a quadratic the three candidates coincide with it, so each
    beta_r is sum_{l=1,2} h^{2l-1} int_cell (p^(l))^2 of that quadratic; the
    oracle's indicators, read back through the weights it forms, must match."""
    rng = np.random.default_rng(W.SEED + 63)
    for _ in range(20):
        widths = rng.uniform(0.5, 2.0, size=5)
        f = np.concatenate([[0.0], np.cumsum(widths)])
        c = rng.normal(size=3)
        avgs = [poly_avg(c, f[t], f[t + 1]) for t in range(5)]
        betas = oracle.weno5_nonuniform_betas(widths, np.asarray(avgs))
        a, b, h = f[2], f[3], widths[2]
        # p' = c1 + 2 c2 x, p'' = 2 c2: integrals in closed form
        i1 = (c[1] ** 2 * (b - a) + 2 * c[1] * c[2] * (b ** 2 - a ** 2) + 4 * c[2] ** 2 * (b ** 3 - a ** 3) / 3)
        i2 = 4 * c[2] ** 2 * (b - a)
        want = h * i1 + h ** 3 * i2
        for beta in betas:
            assert beta == pytest.approx(want, rel=1e-10, abs=1e-13)


@pytest.mark.slow
def test_fifth_order_on_a_stretched_grid():
    def err(n):
        spec, w = W.sine_advection_1d(n, stretch=0.5)
        h = np.diff(spec.faces[0])
        dt0 = min(0.4 * h.min() / (1.0 + math.sqrt(1.4)), 2.0 * h.min() ** (5.0 / 3.0))
        nsteps = int(math.ceil(0.25 / dt0))
        q, t, st = oracle.run(spec, oracle.prim_to_cons_field(spec, w), nsteps, dt=0.25 / nsteps)
        assert st == oracle.OK
        rho = (q[0] + q[1])[spec.interior[1:]].reshape(-1)
        return np.abs(rho - W.sine_cell_averages(spec, t)).mean()
    e = [err(n) for n in (32, 64, 128)]
    order = math.log2(e[1] / e[2])
    assert order >= 4.3, e


def test_conservation_on_a_stretched_periodic_box():
    spec, w = W.random_smooth_periodic(2, 20)
    faces = (W.tanh_faces(20, depth=0.5), W.tanh_faces(20, centre=0.3, depth=0.4), None)
    spec = dataclasses.replace(spec, faces=faces)
    vol = np.outer(np.diff(faces[1]), np.diff(faces[0]))
    q0 = oracle.prim_to_cons_field(spec, w)
    q, _, st = oracle.run(spec, q0, 50, cfl=0.3)
    assert st == oracle.OK
    I = spec.interior[1:]
    for v in range(spec.nvar - 1):
        m0, m1 = (q0[v][I][0] * vol).sum(), (q[v][I][0] * vol).sum()
        scale = (np.abs(q0[v][I][0]) * vol).sum()
        assert abs(m1 - m0) <= 1e-13 * scale, v


def test_cfl_step_uses_the_smallest_cell_crossing_time():
    spec, w = W.bubble_collapse_3d(n=12, stretch=0.6)
    q = oracle.prim_to_cons_field(spec, w)
    _, t, st = oracle.run(spec, q, 1, cfl=0.3)
    assert st == oracle.OK
    wp = w[spec.interior]
    rho = wp[0] + wp[1]
    g1, g2 = 1 / (4.4 - 1), 1 / (1.4 - 1)
    Gam = wp[6] * g1 + (1 - wp[6]) * g2
    Pi = wp[6] * 4.4 * 6e8 / 3.4
    c = np.sqrt(((Gam + 1) * wp[5] + Pi) / (Gam * rho))
    hs = [np.diff(spec.faces[d]) for d in range(3)]
    m = min((hs[0][None, None, :] / (np.abs(wp[2]) + c)).min(), (hs[1][None, :, None] / (np.abs(wp[3]) + c)).min(),
            (hs[2][:, None, None] / (np.abs(wp[4]) + c)).min())
    assert t == pytest.approx(0.3 * m, rel=1e-13)
