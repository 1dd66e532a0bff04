"""What the trained indicator gains over WENO5 alone.

A network is trained on the GPU by the library's own kernels on samples
harvested from FP64 runs (the two-fluid shock tube, the bubble collapse, and
an advected smooth density wave), then:

  * on a smooth flow (the advected sine, exact solution known) the routed
    scheme takes the linear fifth-order stencil almost everywhere and its
    error is several times below WENO5-JS's, whose weights leave the ideal
    ones near the wave's extrema;
  * on the water/air shock tube (exact two-stiffened-gas solution known) it
    keeps WENO5 at the discontinuities: the run stays physical and its
    density error stays close to WENO5's.
"""
import sys

import numpy as np
import pytest
import torch

from exact_riemann import ExactRiemann, Side, mixture_gas
from paper_2305_09163_amd import mfc
from paper_2305_09163_amd import train_indicator as TI
from paper_2305_09163_amd import workloads as W

pytestmark = pytest.mark.gpu
TAU = 0.5


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def trained():
    tube = W.shock_tube_1d(400)
    bub = W.bubble_collapse_3d(n=32)
    runs = [(tube[0], tube[1], list(range(0, 201, 20)), 0.4), (bub[0], bub[1], [0, 5, 10], 0.3)]
    for n in (32, 64, 128):
        sine = W.sine_advection_1d(n)
        runs.append((sine[0], sine[1], [0, n // 4], 0.4))
    X, Y = TI.harvest_runs(runs, log=say)
    params, hist = TI.train(X, Y, steps=1500, batch=4096, seed=1, log=say, log_every=300)
    ev = TI.evaluate(params, X, Y, TAU)
    say(f"[gain] training set {int(Y.numel())} samples: {ev}")
    assert hist[-1][1] < 0.6 * hist[0][1]
    return params


def run(spec, w, nsteps, params=None, cfl=0.0, dt=0.0):
    recon = mfc.MFC_RECON_WENO5 if params is None else mfc.MFC_RECON_LEARNED
    s = mfc.Solver(spec, recon=recon)
    if params is not None:
        s.set_indicator(params, TAU)
    q = s.state_from_prim(w)
    s.run(q, nsteps, cfl=cfl, dt=dt)
    s.check()
    t, _ = s.time()
    return q.cpu().numpy(), t


def test_smooth_flow_error_drops(trained):
    n, t_end = 64, 0.25
    spec, w = W.sine_advection_1d(n)
    dx = spec.dx[0]
    nsteps = int(np.ceil(t_end / min(0.4 * dx / 2.2, 2.0 * dx ** (5.0 / 3.0))))  # RK3 error below spatial
    errs = {}
    for name, p in (("weno5", None), ("learned", trained)):
        q, t = run(spec, w, nsteps, p, dt=t_end / nsteps)
        rho = (q[0] + q[1])[0, 0, 3:-3]
        errs[name] = np.abs(rho - W.sine_cell_averages(spec, t)).mean()
    say(f"[gain] advected sine n={n}: L1 error WENO5 {errs['weno5']:.3e}, learned {errs['learned']:.3e} "
        f"({errs['weno5'] / errs['learned']:.1f}x lower)")
    assert errs["learned"] < 0.5 * errs["weno5"]


def test_shock_tube_stays_close_to_weno(trained):
    spec, w = W.shock_tube_1d(400)
    gL = mixture_gas(1 - 1e-6, spec.gamma, spec.pi_inf)
    gR = mixture_gas(1e-6, spec.gamma, spec.pi_inf)
    rL = (1 - 1e-6) * 1000.0 + 1e-6 * 50.0
    rR = 1e-6 * 1000.0 + (1 - 1e-6) * 50.0
    ex = ExactRiemann(Side(rL, 0.0, 1e9, *gL), Side(rR, 0.0, 1e5, *gR))
    errs = {}
    for name, p in (("weno5", None), ("learned", trained)):
        q, t = run(spec, w, 200, p, cfl=0.4)
        sub = 64
        xs = spec.lo[0] + (np.arange(400 * sub) + 0.5) * spec.dx[0] / sub
        rho_ex = ex.sample((xs - 0.7) / t)[0].reshape(400, sub).mean(1)
        rho = (q[0] + q[1])[0, 0, 3:-3]
        errs[name] = np.abs(rho - rho_ex).sum() / np.abs(rho_ex).sum()
    say(f"[gain] shock tube: L1 density error WENO5 {errs['weno5']:.3e}, learned {errs['learned']:.3e}")
    assert errs["learned"] < 1.25 * errs["weno5"]
