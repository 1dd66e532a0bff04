"""FP64 CPU oracle of the five-equation WENO5/HLLC/SSP-RK3 right-hand side.

TEST INFRASTRUCTURE ONLY: this package is the reference the GPU library is
checked against.  Only the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import it; the GPU library never does, and this
package imports nothing from the GPU library.

The arithmetic lives in ``mfc_oracle.c`` (plain C, built with
``gcc -O2 -ffp-contract=off``); this module only marshals numpy arrays into
it.  Grid arguments are any object with the attributes ``ndim``, ``n``,
``dx``, ``gamma``, ``pi_inf``, ``bc`` and ``weno_eps``.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mfc_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_LIB_OMP_PATH = os.path.join(_HERE, "liboracle_omp.so")
_LIB_FMA_PATH = os.path.join(_HERE, "liboracle_fma.so")
_lib = None
_lib_omp = None
_lib_fma = None
_threaded = False
_contracted = False

OK = 0
E_NONPHYSICAL = -4


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction), once
    plain and once with OpenMP (the same source: its pragmas spread the
    pencils of a sweep over threads; results are bitwise the same).  A third
    build of the same source lets the compiler contract a*b + c into fused
    multiply-adds: another valid rounding order of the same arithmetic, which
    the parity tests use to measure how far rounding alone moves a result."""
    builds = ((_LIB_PATH, ["-ffp-contract=off"]), (_LIB_OMP_PATH, ["-ffp-contract=off", "-fopenmp"]),
              (_LIB_FMA_PATH, ["-ffp-contract=fast", "-mfma"]))
    for path, extra in builds:
        if force or not os.path.exists(path):
            tmp = "%s.%d.tmp" % (path, os.getpid())   # parallel test workers may build at once
            subprocess.run(["gcc", "-O2", "-fno-fast-math", "-std=c99", "-fPIC", "-shared",
                            *extra, "-o", tmp, _SRC, "-lm"], check=True)
            os.replace(tmp, path)
    return _LIB_PATH


_D = ctypes.POINTER(ctypes.c_double)


class _Grid(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int * 3), ("dx", ctypes.c_double * 3),
                ("gamma", ctypes.c_double * 2), ("pi_inf", ctypes.c_double * 2), ("bc", ctypes.c_int * 6),
                ("weno_eps", ctypes.c_double), ("recon", ctypes.c_int),
                ("smooth", ctypes.POINTER(ctypes.c_ubyte)), ("model", ctypes.c_int), ("faces", _D * 3)]


@contextlib.contextmanager
def threaded():
    """Run the oracle calls inside the block on the OpenMP build (as many
    threads as OpenMP gives, OMP_NUM_THREADS or all cores); yields that
    number."""
    global _threaded
    prev = _threaded
    _threaded = True
    try:
        yield lib().ora_threads()
    finally:
        _threaded = prev


@contextlib.contextmanager
def contracted():
    """Run the oracle calls inside the block on the build with fused
    multiply-add contraction (single-threaded)."""
    global _contracted
    prev = _contracted
    _contracted = True
    try:
        yield
    finally:
        _contracted = prev


def lib():
    global _lib, _lib_omp, _lib_fma
    if _contracted:
        if _lib_fma is None:
            if not os.path.exists(_LIB_FMA_PATH) or os.path.getmtime(_SRC) > os.path.getmtime(_LIB_FMA_PATH):
                build(force=True)
            _lib_fma = _load(_LIB_FMA_PATH)
        return _lib_fma
    if _threaded:
        if _lib_omp is None:
            if not os.path.exists(_LIB_OMP_PATH) or os.path.getmtime(_SRC) > os.path.getmtime(_LIB_OMP_PATH):
                build(force=True)
            _lib_omp = _load(_LIB_OMP_PATH)
        return _lib_omp
    if _lib is None:
        path = os.environ.get("MFC_ORACLE_LIB")  # a deliberately broken build, for mutation tests
        if not path:
            path = _LIB_PATH
            if not os.path.exists(path) or os.path.getmtime(_SRC) > os.path.getmtime(path):
                build(force=True)   # missing, or older than its source
        _lib = _load(path)
    return _lib


def _load(path):
    L = ctypes.CDLL(path)
    G = ctypes.POINTER(_Grid)
    sig = {
        "ora_nvar": (ctypes.c_int, [ctypes.c_int]),
        "ora_padded_cells": (ctypes.c_int64, [G]),
        "ora_mixture": (None, [G, ctypes.c_double, _D, _D]),
        "ora_sound_speed2": (ctypes.c_double, [G, ctypes.c_double, ctypes.c_double, ctypes.c_double]),
        "ora_kapila_K": (ctypes.c_double, [G, _D]),
        "ora_cbc_cell": (None, [G, ctypes.c_int, ctypes.c_int, _D, _D, _D]),
        "ora_one_sided_coef": (None, [G, ctypes.c_int, ctypes.c_int, _D]),
        "ora_prim_to_cons": (None, [G, _D, _D]),
        "ora_cons_to_prim": (ctypes.c_int, [G, _D, _D]),
        "ora_weno5": (None, [_D, ctypes.c_double, _D, _D, _D]),
        "ora_linear5": (None, [_D, _D, _D]),
        "ora_weno3": (None, [_D, ctypes.c_double, _D, _D]),
        "ora_weno5_nonuniform_cell": (None, [_D, _D, ctypes.c_double, _D, _D]),
        "ora_weno5_nonuniform_betas": (None, [_D, _D, _D]),
        "ora_hllc": (ctypes.c_int, [G, ctypes.c_int, _D, _D, _D, _D]),
        "ora_fill_ghosts": (ctypes.c_int, [G, _D]),
        "ora_rhs": (ctypes.c_int, [G, _D, _D]),
        "ora_rk3_combine": (ctypes.c_int, [ctypes.c_int, ctypes.c_int64, _D, _D, _D, ctypes.c_double, _D]),
        "ora_max_wavespeed": (ctypes.c_int, [G, _D, _D]),
        "ora_rk3_step": (ctypes.c_int, [G, _D, ctypes.c_double]),
        "ora_run": (ctypes.c_int, [G, _D, ctypes.c_int, ctypes.c_double, ctypes.c_double, _D]),
        "ora_prim_to_cons_field": (ctypes.c_int, [G, _D, _D]),
        "ora_cons_to_prim_field": (ctypes.c_int, [G, _D, _D]),
        "ora_threads": (ctypes.c_int, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    return L


RECON_WENO5, RECON_LINEAR, RECON_MASK, RECON_WENO3, RECON_FIRST = 0, 1, 2, 3, 4
MODEL_ALLAIRE, MODEL_KAPILA = 0, 1


def grid(spec, recon: int = RECON_WENO5, smooth=None) -> _Grid:
    """C grid descriptor.  recon RECON_MASK needs `smooth`, a uint8 array
    [ndim, *padded shape] (kept alive by the caller while the grid is used)."""
    g = _Grid()
    g.recon = recon
    if recon == RECON_MASK:
        assert smooth is not None and smooth.dtype == np.uint8 and smooth.flags["C_CONTIGUOUS"]
        assert smooth.shape == (spec.ndim,) + spec.shape[1:]
        g.smooth = smooth.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte))
    g.ndim = spec.ndim
    for d in range(3):
        g.n[d] = spec.n[d] if d < spec.ndim else 1
        g.dx[d] = spec.dx[d]
    g.gamma[0], g.gamma[1] = spec.gamma
    g.pi_inf[0], g.pi_inf[1] = spec.pi_inf
    for f in range(6):
        g.bc[f] = spec.bc[f]
    g.weno_eps = spec.weno_eps
    g.model = getattr(spec, "model", MODEL_ALLAIRE)
    g._keep = []
    for d in range(3):
        f = spec.face_coords(d) if hasattr(spec, "face_coords") else None
        if f is not None:
            assert f.shape == (spec.n[d] + 1,) and np.all(np.diff(f) > 0)
            g._keep.append(f)
            g.faces[d] = f.ctypes.data_as(_D)
    return g


def _ptr(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _arr(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# --- per-cell / per-face building blocks ---------------------------------

def mixture(spec, alpha1: float):
    G, P = ctypes.c_double(), ctypes.c_double()
    lib().ora_mixture(ctypes.byref(grid(spec)), alpha1, ctypes.byref(G), ctypes.byref(P))
    return G.value, P.value


def sound_speed2(spec, rho: float, p: float, alpha1: float) -> float:
    return lib().ora_sound_speed2(ctypes.byref(grid(spec)), rho, p, alpha1)


def prim_to_cons(spec, w):
    w = _arr(w)
    q = np.empty_like(w)
    lib().ora_prim_to_cons(ctypes.byref(grid(spec)), _ptr(w), _ptr(q))
    return q


def cons_to_prim(spec, q):
    q = _arr(q)
    w = np.empty_like(q)
    st = lib().ora_cons_to_prim(ctypes.byref(grid(spec)), _ptr(q), _ptr(w))
    return w, st


def weno5(s, eps: float = 1e-6):
    """(value at x_{i+1/2}, value at x_{i-1/2}, max |omega - d|) from 5 cell averages."""
    s = _arr(s)
    a, b, dev = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    lib().ora_weno5(_ptr(s), eps, ctypes.byref(a), ctypes.byref(b), ctypes.byref(dev))
    return a.value, b.value, dev.value


def weno3(s, eps: float = 1e-6):
    """(value at x_{i+1/2}, value at x_{i-1/2}) from 3 cell averages."""
    s = _arr(s)
    a, b = ctypes.c_double(), ctypes.c_double()
    lib().ora_weno3(_ptr(s), eps, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def weno5_nonuniform(widths, s, eps: float = 1e-6):
    """(value at x_{i+1/2}, value at x_{i-1/2}) of cell i from the widths and
    averages of cells i-2 .. i+2 (non-uniform WENO5)."""
    widths, s = _arr(widths), _arr(s)
    a, b = ctypes.c_double(), ctypes.c_double()
    lib().ora_weno5_nonuniform_cell(_ptr(widths), _ptr(s), eps, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def weno5_nonuniform_betas(widths, s):
    widths, s = _arr(widths), _arr(s)
    out = np.empty(3)
    lib().ora_weno5_nonuniform_betas(_ptr(widths), _ptr(s), _ptr(out))
    return out


def linear5(s):
    s = _arr(s)
    a, b = ctypes.c_double(), ctypes.c_double()
    lib().ora_linear5(_ptr(s), ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


def hllc(spec, direction: int, wL, wR):
    """(flux[nv], face velocity, status) at a face normal to `direction`."""
    wL, wR = _arr(wL), _arr(wR)
    F = np.empty(spec.nvar)
    uf = ctypes.c_double()
    st = lib().ora_hllc(ctypes.byref(grid(spec)), direction, _ptr(wL), _ptr(wR), _ptr(F), ctypes.byref(uf))
    return F, uf.value, st


# --- whole-grid operations ------------------------------------------------

def prim_to_cons_field(spec, w):
    w = _arr(w)
    assert w.shape == spec.shape
    q = np.empty_like(w)
    lib().ora_prim_to_cons_field(ctypes.byref(grid(spec)), _ptr(w), _ptr(q))
    return q


def kapila_K(spec, w_cell):
    """K of the Kapila volume-fraction equation for one cell's primitive
    vector (nvar values)."""
    w = _arr(w_cell)
    assert w.shape == (spec.nvar,)
    return lib().ora_kapila_K(ctypes.byref(grid(spec)), _ptr(w))


def cbc_cell(spec, d: int, side: int, w_cell, dwdx):
    """Normal-direction conservative time derivative of a characteristic
    (non-reflecting) boundary cell along d (side 0 low, 1 high) from its
    primitives and their normal derivative."""
    w, dw = _arr(w_cell), _arr(dwdx)
    out = np.empty(spec.nvar)
    lib().ora_cbc_cell(ctypes.byref(grid(spec)), d, side, _ptr(w), _ptr(dw), _ptr(out))
    return out


def one_sided_coef(spec, d: int, side: int):
    """Coefficients of the second-order one-sided derivative along d at the
    centre of the boundary cell of face `side` (0 low, 1 high), for the
    values of that cell and the next two cells into the domain."""
    out = np.empty(3)
    lib().ora_one_sided_coef(ctypes.byref(grid(spec)), d, side, _ptr(out))
    return out


def cons_to_prim_field(spec, q):
    q = _arr(q)
    assert q.shape == spec.shape
    w = np.empty_like(q)
    st = lib().ora_cons_to_prim_field(ctypes.byref(grid(spec)), _ptr(q), _ptr(w))
    return w, st


def fill_ghosts(spec, q):
    """Returns a copy of q with the ghost face slabs filled."""
    q = _arr(q).copy()
    assert q.shape == spec.shape
    lib().ora_fill_ghosts(ctypes.byref(grid(spec)), _ptr(q))
    return q


def rhs(spec, q, recon: int = RECON_WENO5, smooth=None):
    """(dq/dt on interior cells (ghost entries zero), status); q must have
    ghosts filled.  recon/smooth select the reconstruction (see grid)."""
    q = _arr(q)
    assert q.shape == spec.shape
    out = np.zeros_like(q)
    if smooth is not None:
        smooth = np.ascontiguousarray(smooth, dtype=np.uint8)
    st = lib().ora_rhs(ctypes.byref(grid(spec, recon, smooth)), _ptr(q), _ptr(out))
    return out, st


def rk3_combine(stage: int, q0, qs, L, dt: float):
    q0, qs, L = _arr(q0), _arr(qs), _arr(L)
    out = np.empty_like(q0)
    st = lib().ora_rk3_combine(stage, q0.size, _ptr(q0), _ptr(qs), _ptr(L), dt, _ptr(out))
    assert st == OK
    return out


def max_wavespeed(spec, q):
    q = _arr(q)
    s = ctypes.c_double()
    st = lib().ora_max_wavespeed(ctypes.byref(grid(spec)), _ptr(q), ctypes.byref(s))
    return s.value, st


def rk3_step(spec, q, dt: float):
    """(q after one SSP-RK3 step of size dt, status)."""
    q = _arr(q).copy()
    st = lib().ora_rk3_step(ctypes.byref(grid(spec)), _ptr(q), dt)
    return q, st


def run(spec, q, nsteps: int, cfl: float = 0.0, dt: float = 0.0, recon: int = RECON_WENO5):
    """(q after nsteps steps, total time, status); CFL time step if cfl > 0.
    recon RECON_LINEAR runs the linear fifth-order scheme everywhere, RECON_WENO3
    WENO3 and RECON_FIRST the first-order (cell-value) reconstruction."""
    assert recon in (RECON_WENO5, RECON_LINEAR, RECON_WENO3, RECON_FIRST)
    q = _arr(q).copy()
    t = ctypes.c_double()
    st = lib().ora_run(ctypes.byref(grid(spec, recon)), _ptr(q), nsteps, cfl, dt, ctypes.byref(t))
    return q, t.value, st
