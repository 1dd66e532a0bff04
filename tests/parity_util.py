"""Error norms used by the parity tests: this module's reading of "relative
L-infinity / L1", stated below.

States: per variable, the maximum (or sum) of |a - b| over interior cells
divided by the same norm of the reference b.  The momentum components are
one vector, so they share one scale (the largest |b| over all components):
a component that is zero in the reference (a 1D problem, a fluid at rest)
is measured against the momentum that does exist, never against itself.

A momentum that is small against its natural size (a fluid that starts
at rest) is measured against the acoustic momentum scale rho_max * c_max
of the initial state (`acoustic_floor`): in water the pressure recovery
p = (rho E - rho|u|^2/2 - Pi)/Gamma amplifies one rounding of rho E by
Pi/(Gamma p) ~ 3e3 at 1e6 Pa, so rounding differences of an equally
correct evaluation order reach the momentum at that level.

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
