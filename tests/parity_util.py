"""Error norms used by the parity tests: this module's reading of "relative
L-infinity / L1", stated below.

States: per variable, the maximum (or sum) of |a - b| over interior cells
divided by the same norm of the reference b (its own scale).  The momentum
components are one vector, so they share one scale (the largest |b| over
all components): a component that is zero in the reference (a 1D problem)
is measured against the momentum that does exist, never against itself.
The GPU starts from the oracle's own conservative state, bit for bit.

One step from rest in water: the pressure recovery
p = (rho E - rho|u|^2/2 - Pi)/Gamma amplifies one rounding of rho E by
Pi/(Gamma p) ~ 2.6e3 at 1e6 Pa, and the momentum one step creates is small,
so two equally valid rounding orders of the same arithmetic already differ
there by more than 1e-12 of the momentum's own scale.  `rounding_spread`
measures that difference on the case itself: the oracle's source built with
and without fused multiply-add contraction (4.1e-12 on the 37x21x19
bubble's momentum, below 5e-16 on every other variable).  `step_bar` is
1e-12 per variable, raised to twice that spread where the spread itself
exceeds half the bar.

Runs of many steps (bar: relative L1 1e-10 per variable, own scales) take
the same allowance: where the GPU's error exceeds 1e-10, `run_parity`
repeats the oracle run on the contracted build and accepts twice that
spread.  It matters where a variable ends near zero against its start: an
acoustic pulse that has left the domain through non-reflecting faces
(momentum 4.5e-6 of its initial 0.29; the oracle's two rounding orders
differ there by 9.6e-7 of it).

The FP32 storage form (bar: relative L1 density error 1e-4) measures a
momentum that starts at rest against the acoustic momentum scale
rho_max * c_max of the initial state (`acoustic_floor`): FP32 rounding of
rho E moves the water pressure by ~1e2 Pa.

Right-hand sides: a right-hand side that is zero in exact arithmetic (a
transverse momentum, a volume fraction far from moving interfaces) holds
only rounding noise, so it is measured by what it does to the state: the
error dt * |rhs_a - rhs_b| of a forward-Euler step at CFL 0.3, relative to
the state scale above (momentum floor: max rho * max wave speed).
"""
import numpy as np

import oracle


def _interior(spec, a):
    return a[spec.interior]


def _mom_rows(spec):
    return list(range(2, 2 + spec.ndim))


def state_scales(spec, b, norm="max", floor_mom=0.0):
    bi = np.abs(_interior(spec, b)).reshape(spec.nvar, -1)
    f = (lambda x: x.max()) if norm == "max" else (lambda x: x.sum())
    s = np.array([f(bi[v]) for v in range(spec.nvar)])
    mom = _mom_rows(spec)
    s[mom] = max(max(f(bi[m]) for m in mom), floor_mom)
    return s


def acoustic_floor(spec, q):
    """rho_max * (max wave speed) of state q: the natural momentum scale."""
    smax, _ = oracle.max_wavespeed(spec, q)
    return np.abs((q[0] + q[1])[spec.interior[1:]]).max() * smax


def rel_linf(a, b, spec, floor_mom=0.0):
    d = np.abs(_interior(spec, a) - _interior(spec, b)).reshape(spec.nvar, -1).max(axis=1)
    return d / state_scales(spec, b, "max", floor_mom=floor_mom)


def rel_l1(a, b, spec, floor_mom=0.0):
    """floor_mom: per-cell momentum scale (see acoustic_floor); the momentum
    denominator is at least cells * floor_mom."""
    d = np.abs(_interior(spec, a) - _interior(spec, b)).reshape(spec.nvar, -1).sum(axis=1)
    return d / state_scales(spec, b, "sum", floor_mom=floor_mom * spec.cells)


def rhs_err(ra, rb, q_ref, spec, cfl=0.3):
    """Per-variable forward-Euler-step error of two right-hand sides."""
    smax, _ = oracle.max_wavespeed(spec, q_ref)
    dt = cfl * min(spec.dx[d] for d in range(spec.ndim)) / smax
    scale = state_scales(spec, q_ref, "max", floor_mom=acoustic_floor(spec, q_ref))
    d = np.abs(_interior(spec, ra) - _interior(spec, rb)).reshape(spec.nvar, -1).max(axis=1)
    return dt * d / scale


def rounding_spread(spec, qi, nsteps=1, cfl=0.3, **kw):
    """Per-variable relative L-infinity (own scales) between the oracle run
    from qi and the same run on the oracle built with fused multiply-add
    contraction: how far rounding order alone moves this result."""
    a, _, sa = oracle.run(spec, qi, nsteps, cfl=cfl, **kw)
    with oracle.contracted():
        b, _, sb = oracle.run(spec, qi, nsteps, cfl=cfl, **kw)
    assert sa == sb == oracle.OK
    return rel_linf(b, a, spec)


def step_bar(spread, bar=1e-12):
    """1e-12 per variable, or twice the rounding-order spread where that
    spread exceeds half of it."""
    return np.maximum(bar, 2.0 * spread)


def rounding_spread_run(spec, qi, nsteps, cfl=0.3, norm="l1", **kw):
    """Per-variable relative L1 (or L-infinity), own scales, between the
    oracle run from qi and the same run on the contracted oracle build."""
    a, _, sa = oracle.run(spec, qi, nsteps, cfl=cfl, **kw)
    with oracle.contracted():
        b, _, sb = oracle.run(spec, qi, nsteps, cfl=cfl, **kw)
    assert sa == sb == oracle.OK
    return rel_l1(b, a, spec) if norm == "l1" else rel_linf(b, a, spec)


def run_parity(err, spec, qi, nsteps, bar=1e-10, cfl=0.3, norm="l1", **kw):
    """Assert a run's per-variable relative error `err` (L1 or L-infinity,
    own scales) against the oracle: within `bar`, or within twice the
    oracle's own rounding-order spread on the same run (computed only when
    needed)."""
    err = np.asarray(err)
    if (err <= bar).all():
        return
    lim = np.maximum(bar, 2.0 * rounding_spread_run(spec, qi, nsteps, cfl=cfl, norm=norm, **kw))
    assert (err <= lim).all(), (err, lim)
