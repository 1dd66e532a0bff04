"""Seeded synthetic inputs: grid descriptions and initial primitive states.

This module builds the grids and the initial conditions of the two-fluid
(water/air) workloads that stand in for the paper's air/water problems: a 1D
two-fluid shock tube, a 3D bubble collapse, a 3D bubble cloud struck by a
pressure step and 2D shock-droplet runs, plus the smooth, periodic and
interface-advection states that the accuracy tests use.

It holds none of the method's arithmetic.  Every generator returns
*primitive* fields on the full padded grid (ghost cells included, evaluated
at their own cell centres) in the state ordering
``[alpha1*rho1, alpha2*rho2, u_1 .. u_ndim, p, alpha1]``; each consumer
converts them to conservative variables with its own equation of state.
Random numbers come from ``numpy.random.default_rng(SEED + k)``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED = 230509163
NG = 3  # ghost layers per side on active dimensions

# Stiffened-gas parameters of the two fluids (fluid 1 = water, fluid 2 = air).
WATER = dict(gamma=4.4, pi_inf=6.0e8)
AIR = dict(gamma=1.4, pi_inf=0.0)
ALPHA_MIN = 1.0e-6


@dataclasses.dataclass
class GridSpec:
    """Uniform Cartesian grid and fluid parameters of one run."""

    ndim: int
    n: tuple                      # interior cells (nx, ny, nz); 1 on inactive dims
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)
    gamma: tuple = (WATER["gamma"], AIR["gamma"])
    pi_inf: tuple = (WATER["pi_inf"], AIR["pi_inf"])
    bc: tuple = (0, 0, 0, 0, 0, 0)  # x-,x+,y-,y+,z-,z+: 0 extrapolation, 1 periodic
    weno_eps: float = 1.0e-6
    model: int = 0                  # 0 Allaire five-equation model, 1 Kapila (with K div(u))
    faces: tuple = None             # non-uniform grid: per dimension the n_d + 1 interior face
                                    # coordinates (None for a uniform dimension), or None

    def __post_init__(self):
        n = list(self.n) + [1] * (3 - len(self.n))
        for d in range(self.ndim, 3):
            n[d] = 1
        self.n = tuple(int(v) for v in n)

    @property
    def nvar(self) -> int:
        return 4 + self.ndim

    @property
    def dx(self) -> tuple:
        return tuple((self.hi[d] - self.lo[d]) / self.n[d] if d < self.ndim else 1.0 for d in range(3))

    def padded(self, d: int) -> int:
        return self.n[d] + 2 * NG if d < self.ndim else 1

    @property
    def shape(self) -> tuple:
        """Array shape (nvar, pz, py, px) of a state on this grid."""
        return (self.nvar, self.padded(2), self.padded(1), self.padded(0))

    @property
    def interior(self) -> tuple:
        """Slices selecting interior cells of a (nvar, pz, py, px) array."""
        s = [slice(None)]
        for d in (2, 1, 0):
            g = NG if d < self.ndim else 0
            s.append(slice(g, g + self.n[d]))
        return tuple(s)

    @property
    def cells(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    def face_coords(self, d: int):
        """Interior face coordinates along d of a non-uniform dimension, else None."""
        if self.faces is None or d >= self.ndim or self.faces[d] is None:
            return None
        return np.ascontiguousarray(self.faces[d], dtype=np.float64)

    def centres(self, d: int) -> np.ndarray:
        """Cell-centre coordinates along dimension d, ghost cells included
        (ghost cells of a non-uniform dimension continue its end widths)."""
        if d >= self.ndim:
            return np.array([0.5 * (self.lo[d] + self.hi[d])])
        f = self.face_coords(d)
        if f is None:
            i = np.arange(-NG, self.n[d] + NG)
            return self.lo[d] + (i + 0.5) * self.dx[d]
        c = 0.5 * (f[1:] + f[:-1])
        lo = c[0] - (np.arange(NG, 0, -1)) * (f[1] - f[0])
        hi = c[-1] + np.arange(1, NG + 1) * (f[-1] - f[-2])
        return np.concatenate([lo, c, hi])

    def mesh(self):
        """Broadcastable (z, y, x) coordinate arrays of shape (pz, py, px)."""
        z = self.centres(2)[:, None, None]
        y = self.centres(1)[None, :, None]
        x = self.centres(0)[None, None, :]
        return x, y, z


def _assemble(spec: GridSpec, alpha1, rho1, rho2, vel, p) -> np.ndarray:
    """Stack primitive fields into a (nvar, pz, py, px) float64 array."""
    shape = spec.shape[1:]
    w = np.empty(spec.shape, dtype=np.float64)
    a1 = np.broadcast_to(alpha1, shape)
    w[0] = a1 * np.broadcast_to(rho1, shape)
    w[1] = (1.0 - a1) * np.broadcast_to(rho2, shape)
    for m in range(spec.ndim):
        w[2 + m] = np.broadcast_to(vel[m], shape)
    w[2 + spec.ndim] = np.broadcast_to(p, shape)
    w[3 + spec.ndim] = a1
    return w


def _smooth_step(s, width):
    """0 for s << -width, 1 for s >> width: the tanh profile of a smeared interface."""
    return 0.5 * (1.0 + np.tanh(s / width))


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def shock_tube_1d(n: int = 400):
    """1D water/air shock tube on [0, 1]: water (rho 1000, p 1e9) for x < 0.7,
    air (rho 50, p 1e5) for x > 0.7, alpha1 = 1 - 1e-6 / 1e-6, u = 0,
    extrapolation boundaries."""
    spec = GridSpec(ndim=1, n=(n,))
    x, _, _ = spec.mesh()
    water = x < 0.7
    alpha1 = np.where(water, 1.0 - ALPHA_MIN, ALPHA_MIN)
    p = np.where(water, 1.0e9, 1.0e5)
    w = _assemble(spec, alpha1, 1000.0, 50.0, [0.0], p)
    return spec, w


def _real_sph_harm_sum(theta, phi, coeffs, lmax):
    """S(theta, phi) = sum_{l=2..lmax} sum_{m=-l..l} a_lm Y_lm with real,
    orthonormal spherical harmonics built from associated Legendre functions."""
    from scipy.special import lpmv

    ct = np.cos(theta)
    s = np.zeros(np.broadcast(theta, phi).shape)
    k = 0
    for l in range(2, lmax + 1):
        for m in range(-l, l + 1):
            am = abs(m)
            norm = math.sqrt((2 * l + 1) / (4 * math.pi) * math.factorial(l - am) / math.factorial(l + am))
            leg = lpmv(am, l, ct)
            if m > 0:
                ang = math.sqrt(2.0) * np.cos(am * phi)
            elif m < 0:
                ang = math.sqrt(2.0) * np.sin(am * phi)
            else:
                ang = 1.0
            s = s + coeffs[k] * norm * leg * ang
            k += 1
    return s


def bubble_collapse_3d(n: int = 128, seed_offset: int = 2, noise: float = 0.01, lmax: int = 8,
                       radius: float = 0.1, centre=(0.5, 0.5, 0.5), p_bubble: float = 1.0e4,
                       p_water: float = 1.0e6, smear_cells: float = 1.0, stretch: float = 0.0):
    """3D air bubble (radius 0.1 at the box centre, p = 1e4) in water at p = 1e6,
    u = 0, on the unit cube.  The bubble surface R(theta, phi) =
    R0 (1 + noise * S / max|S|) carries seeded real spherical-harmonic noise
    (l = 2..8, a_lm ~ N(0, 1)), and the interface is smeared by
    H = (1 + tanh((r - R)/dx))/2; alpha1 = a_min + (1 - 2 a_min) H, and the
    same H blends the pressure.  noise = 0 gives an exactly centred sphere.
    n may be an int (cube) or an (nx, ny, nz) tuple on the same unit cube.
    stretch > 0 refines every dimension around the centre with
    tanh_faces(n_d, depth=stretch) (the smear then uses the finest width)."""
    ns = (n, n, n) if isinstance(n, int) else tuple(n)
    faces = tuple(tanh_faces(ns[d], depth=stretch) for d in range(3)) if stretch > 0.0 else None
    spec = GridSpec(ndim=3, n=ns, faces=faces)
    x, y, z = spec.mesh()
    rx, ry, rz = x - centre[0], y - centre[1], z - centre[2]
    r = np.sqrt(rx * rx + ry * ry + rz * rz)
    if noise > 0.0:
        rng = np.random.default_rng(SEED + seed_offset)
        ncoef = (lmax + 1) ** 2 - 4
        coeffs = rng.standard_normal(ncoef)
        tg = (np.arange(256) + 0.5) * math.pi / 256
        pg = np.arange(512) * 2.0 * math.pi / 512
        smax = np.abs(_real_sph_harm_sum(tg[:, None], pg[None, :], coeffs, lmax)).max()
        # the noise only matters where the tanh profile is not saturated
        # (tanh(x) rounds to +-1 in double precision beyond |x| ~ 19.1)
        rb, (bx, by, bz) = np.broadcast_arrays(r, rx, ry, rz)[0], np.broadcast_arrays(rx, ry, rz)
        near = np.abs(rb - radius) < radius * noise + 20.0 * smear_cells * max(spec.dx)
        theta = np.arccos(np.clip(bz[near] / np.maximum(rb[near], 1e-300), -1.0, 1.0))
        phi = np.arctan2(by[near], bx[near])
        R = np.full(rb.shape, radius)
        R[near] = radius * (1.0 + noise * _real_sph_harm_sum(theta, phi, coeffs, lmax) / smax)
    else:
        R = radius
    h = spec.dx[0] if faces is None else min(np.diff(f).min() for f in faces)
    H = _smooth_step(r - R, smear_cells * h)
    alpha1 = ALPHA_MIN + (1.0 - 2.0 * ALPHA_MIN) * H
    p = p_bubble + (p_water - p_bubble) * H
    w = _assemble(spec, alpha1, 1000.0, 1.2, [0.0, 0.0, 0.0], p)
    return spec, w


def bubble_cloud_3d(n: int = 256, nbubbles: int = 50, seed_offset: int = 3, rmin: float = 0.02,
                    rmax: float = 0.04, gap: float = 0.01, p_ambient: float = 1.0e5,
                    p_step: float = 1.0e7, x_step: float = 0.05):
    """3D cloud of non-overlapping air bubbles (radii U[0.02, 0.04], centres
    U([0.15, 0.95] x [0.05, 0.95]^2), gap >= 0.01) in water at 1e5 Pa, with a
    water slab x < 0.05 at 1e7 Pa: a planar pressure step entering from x = 0.
    Bubble placement depends only on the seed, not on n."""
    rng = np.random.default_rng(SEED + seed_offset)
    centres, radii = [], []
    while len(centres) < nbubbles:
        c = rng.uniform([0.15, 0.05, 0.05], [0.95, 0.95, 0.95])
        r = rng.uniform(rmin, rmax)
        if all(np.linalg.norm(c - c2) >= r + r2 + gap for c2, r2 in zip(centres, radii)):
            centres.append(c)
            radii.append(r)
    spec = GridSpec(ndim=3, n=(n, n, n))
    x, y, z = spec.mesh()
    dist = np.full(np.broadcast(x, y, z).shape, np.inf)
    for c, r in zip(centres, radii):
        dist = np.minimum(dist, np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2) - r)
    H = _smooth_step(dist, spec.dx[0])
    alpha1 = ALPHA_MIN + (1.0 - 2.0 * ALPHA_MIN) * H
    step = _smooth_step(x_step - x, spec.dx[0])
    p = p_ambient + (p_step - p_ambient) * step * np.ones_like(H)
    w = _assemble(spec, alpha1, 1000.0, 1.2, [0.0, 0.0, 0.0], p)
    return spec, w


def normal_shock_air(mach: float, p1: float = 1.0e5, rho1: float = 1.2, gamma: float = 1.4):
    """Post-shock (p, rho, u) of a normal shock of Mach number `mach` moving
    into quiescent ideal gas (Rankine-Hugoniot relations); also the shock speed."""
    m2 = mach * mach
    p2 = p1 * (1.0 + 2.0 * gamma / (gamma + 1.0) * (m2 - 1.0))
    rho2 = rho1 * (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    ws = mach * math.sqrt(gamma * p1 / rho1)
    u2 = ws * (1.0 - rho1 / rho2)
    return p2, rho2, u2, ws


def droplet_shock_2d(n, seed: int, mach: float = 1.5, x_shock: float = 0.1):
    """2D water droplets (1-8, radii U[0.05, 0.15], centres U([0.3, 0.9] x
    [0.1, 0.9]), non-overlapping) in air at 1e5 Pa, struck by a Mach-1.5
    air shock at x = 0.1 moving in +x, on the unit square; n cells per side
    (an int) or (nx, ny)."""
    rng = np.random.default_rng(seed)
    ndrop = int(rng.integers(1, 9))
    centres, radii = [], []
    tries = 0
    while len(centres) < ndrop and tries < 10000:
        tries += 1
        c = rng.uniform([0.3, 0.1], [0.9, 0.9])
        r = rng.uniform(0.05, 0.15)
        if all(np.linalg.norm(c - c2) >= r + r2 for c2, r2 in zip(centres, radii)):
            centres.append(c)
            radii.append(r)
    spec = GridSpec(ndim=2, n=(n, n) if isinstance(n, (int, np.integer)) else tuple(n))
    x, y, _ = spec.mesh()
    dist = np.full(np.broadcast(x, y).shape, np.inf)
    for c, r in zip(centres, radii):
        dist = np.minimum(dist, np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2) - r)
    water = _smooth_step(-dist, max(spec.dx[:2]))  # 1 inside droplets, smeared over the coarser spacing
    alpha1 = ALPHA_MIN + (1.0 - 2.0 * ALPHA_MIN) * water
    p2, rho2, u2, _ = normal_shock_air(mach)
    behind = _smooth_step(x_shock - x, spec.dx[0]) * np.ones_like(water)
    p = 1.0e5 + (p2 - 1.0e5) * behind
    rho_air = 1.2 + (rho2 - 1.2) * behind
    u = u2 * behind
    w = _assemble(spec, alpha1, 1000.0, rho_air, [u, np.zeros_like(u)], p)
    return spec, w


def ensemble_sizes(count: int = 64, seed_offset: int = 5):
    """Seeded uneven square sizes N = 16 * randint(4, 32) in [64, 512]."""
    rng = np.random.default_rng(SEED + seed_offset)
    return [int(16 * v) for v in rng.integers(4, 33, size=count)]


# ---------------------------------------------------------------------------
# States for accuracy and invariant tests
# ---------------------------------------------------------------------------

def ideal_pair():
    """Two fluids that are both the same ideal gas (gamma 1.4, pi 0)."""
    return dict(gamma=(1.4, 1.4), pi_inf=(0.0, 0.0))


def sine_advection_1d(n: int, amplitude: float = 0.2, u: float = 1.0, p: float = 1.0, stretch: float = 0.0):
    """Smooth density wave rho = 1 + 0.2 sin(2 pi x) (as exact cell averages)
    advected at u = 1 with uniform p = 1, periodic on [0, 1]; alpha1 = 0.5 and
    both fluids the same ideal gas, so the exact solution is the translate of
    the initial state.  Each partial density is half the mixture density.
    stretch > 0 puts it on tanh_faces(n, depth=stretch)."""
    faces = (tanh_faces(n, depth=stretch), None, None) if stretch > 0.0 else None
    spec = GridSpec(ndim=1, n=(n,), bc=(1, 1, 0, 0, 0, 0), faces=faces, **ideal_pair())
    xl, xr = _cell_edges(spec)
    k = 2.0 * math.pi
    # exact cell averages (u and p uniform, so the conserved averages follow)
    rho = 1.0 + amplitude * (np.cos(k * xl) - np.cos(k * xr)) / (k * (xr - xl))
    return spec, _assemble(spec, 0.5, rho[None, None, :], rho[None, None, :], [u], p)


def _cell_edges(spec: GridSpec):
    """Left and right x edges of every padded cell along x (ghost cells of a
    periodic dimension are the interior cells one period away)."""
    n = spec.n[0]
    f = spec.face_coords(0)
    if f is None:
        f = spec.lo[0] + np.arange(n + 1) * spec.dx[0]
    L = spec.hi[0] - spec.lo[0]
    i = np.arange(-NG, n + NG)
    j = np.mod(i, n)
    shift = (i - j) // n * L
    return f[j] + shift, f[j + 1] + shift


def sine_cell_averages(spec: GridSpec, t: float, amplitude: float = 0.2, u: float = 1.0):
    """Exact interior cell averages of the translated sine density at time t."""
    xl, xr = _cell_edges(spec)
    xl, xr = xl[NG:-NG] - u * t, xr[NG:-NG] - u * t
    k = 2.0 * math.pi
    return 1.0 + amplitude * (np.cos(k * xl) - np.cos(k * xr)) / (k * (xr - xl))


def interface_advection(ndim: int, n: int, u: float = 100.0, p: float = 1.0e5, width_cells: float = 1.0,
                        direction: int = 0):
    """Periodic water/air slab (water for 0.25 < x_d < 0.75, tanh-smeared)
    advected at uniform velocity u along dimension `direction` in uniform
    pressure p."""
    ns = tuple([n] * ndim)
    spec = GridSpec(ndim=ndim, n=ns, bc=(1, 1, 1, 1, 1, 1))
    coords = spec.mesh()
    xd = coords[direction]
    H = _smooth_step(xd - 0.25, width_cells * spec.dx[direction]) * _smooth_step(0.75 - xd, width_cells * spec.dx[direction])
    alpha1 = ALPHA_MIN + (1.0 - 2.0 * ALPHA_MIN) * H
    vel = [0.0] * ndim
    vel[direction] = u
    return spec, _assemble(spec, alpha1 * np.ones(spec.shape[1:]), 1000.0, 1.2, vel, p)


def uniform_state(ndim: int, n, alpha1: float = 0.4, vel=(37.0, -12.0, 5.0), p: float = 2.0e5):
    """A uniform two-fluid state (extrapolation boundaries): its exact
    right-hand side is zero."""
    spec = GridSpec(ndim=ndim, n=(n,) * ndim if isinstance(n, int) else tuple(n))
    return spec, _assemble(spec, alpha1, 1000.0, 1.2, list(vel[:ndim]), p)


def supersonic_periodic(ndim: int, n: int, mach: float = 2.5, sign: float = 1.0, seed_offset: int = 9):
    """The smooth periodic state of random_smooth_periodic with both fluids
    air-like ideal gases and a uniform velocity of `mach` times the largest
    sound speed added along every direction (sign -1: towards -x, -y, -z),
    so that every face is supersonic and the HLLC flux is one-sided."""
    spec0, w = random_smooth_periodic(ndim, n, seed_offset=seed_offset)
    spec = GridSpec(ndim=ndim, n=spec0.n[:ndim], bc=spec0.bc, **ideal_pair())
    rho = w[0] + w[1]
    p = w[2 + ndim]
    cmax = float(np.sqrt(1.4 * p / rho).max())
    for d in range(ndim):
        w[2 + d] = w[2 + d] + sign * mach * cmax
    return spec, w


def sod_1d(n: int = 100):
    """Sod's problem with both fluids the same ideal gas (gamma 1.4): rho, p =
    (1, 1) for x < 0.5 and (0.125, 0.1) after, u = 0, alpha1 = 0.5."""
    spec = GridSpec(ndim=1, n=(n,), **ideal_pair())
    x, _, _ = spec.mesh()
    left = x < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    return spec, _assemble(spec, 0.5, rho, rho, [np.zeros_like(x)], p)


def tanh_faces(n: int, centre: float = 0.5, width: float = 0.1, depth: float = 0.6, lo: float = 0.0,
               hi: float = 1.0) -> np.ndarray:
    """n + 1 face coordinates on [lo, hi] refined around `centre` by a
    hyperbolic-tangent map: x(s) proportional to s - depth*width*tanh((s - centre)/width)
    for uniform s, so cells near the centre are (1 - depth) times the far
    ones (Sec. 4.1 uses tanh stretching to refine locally)."""
    s = lo + (hi - lo) * np.arange(n + 1) / n
    g = s - depth * width * np.tanh((s - centre) / width)
    return lo + (hi - lo) * (g - g[0]) / (g[-1] - g[0])


def random_smooth_periodic(ndim: int, n: int, seed_offset: int = 7, modes: int = 3):
    """Random smooth periodic state (sums of low Fourier modes) with both
    fluids present everywhere: alpha1 in [0.3, 0.7], densities near water and
    air values, velocities O(10) m/s, pressure around 1e5 Pa."""
    rng = np.random.default_rng(SEED + seed_offset)
    spec = GridSpec(ndim=ndim, n=tuple([n] * ndim), bc=(1, 1, 1, 1, 1, 1))
    coords = spec.mesh()
    shape = spec.shape[1:]

    def field():
        f = np.zeros(shape)
        for _ in range(modes):
            k = rng.integers(1, 3, size=ndim)
            ph = rng.uniform(0, 2 * math.pi)
            arg = ph + sum(2 * math.pi * k[d] * coords[d] for d in range(ndim))
            f = f + rng.uniform(0.2, 1.0) * np.sin(arg)
        return f / modes

    alpha1 = 0.5 + 0.2 * field()
    rho1 = 1000.0 * (1.0 + 0.01 * field())
    rho2 = 1.2 * (1.0 + 0.1 * field())
    vel = [10.0 * field() for _ in range(ndim)]
    p = 1.0e5 * (1.0 + 0.3 * field())
    return spec, _assemble(spec, alpha1, rho1, rho2, vel, p)
