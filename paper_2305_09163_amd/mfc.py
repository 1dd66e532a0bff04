"""Python binding of the C ABI in include/mfc.h (ctypes; argument marshalling only).

Every step of the right-hand side runs in the HIP kernels of ``libmfc.so``;
PyTorch supplies device memory (tensors of the state layout) and the stream.
The binding refuses to run if the library has not been built: there is no
CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("MFC_LIB") or os.path.join(HERE, "libmfc.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mfc.h")

MFC_OK = 0
MFC_E_ARG = -1
MFC_E_NOMEM = -2
MFC_E_HIP = -3
MFC_E_NONPHYSICAL = -4
MFC_E_UNSUPPORTED = -5
MFC_BC_EXTRAP, MFC_BC_PERIODIC, MFC_BC_CHARACTERISTIC = 0, 1, 2
MFC_FP64, MFC_FP32_MIXED = 0, 1
MFC_RECON_WENO5, MFC_RECON_LEARNED, MFC_RECON_WENO3, MFC_RECON_FIRST_ORDER = 0, 1, 2, 3
MFC_KERNEL_FUSED, MFC_KERNEL_STAGED, MFC_KERNEL_SPLIT = 0, 1, 2
MFC_MODEL_ALLAIRE, MFC_MODEL_KAPILA = 0, 1


class MfcError(RuntimeError):
    def __init__(self, status: int, call: str, detail: str):
        super().__init__(f"{call} failed: {status} ({detail})")
        self.status = status


class mfc_grid_desc(ctypes.Structure):
    _fields_ = [("ndim", ctypes.c_int), ("n", ctypes.c_int * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3), ("num_fluids", ctypes.c_int), ("gamma", ctypes.c_double * 2),
                ("pi_inf", ctypes.c_double * 2), ("bc", ctypes.c_int * 6), ("precision", ctypes.c_int),
                ("recon", ctypes.c_int), ("weno_eps", ctypes.c_double), ("kernel", ctypes.c_int),
                ("model", ctypes.c_int), ("faces", ctypes.POINTER(ctypes.c_double) * 3)]


class mfc_batch_tune(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int), ("groups", ctypes.c_int), ("xcd", ctypes.c_int)]


BATCH_SHAPES = ((16, 16), (32, 8), (64, 4))
BATCH_GROUPS_PER_CU = (1, 2, 4)

_lib = None
_VP = ctypes.c_void_p
_SIGNATURES = {
    "mfc_init_grid": [ctypes.POINTER(mfc_grid_desc), ctypes.POINTER(_VP)],
    "mfc_free_grid": [_VP],
    "mfc_state_layout": [_VP, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                         ctypes.POINTER(ctypes.c_int64)],
    "mfc_prim_to_cons": [_VP, _VP, _VP, _VP],
    "mfc_cons_to_prim": [_VP, _VP, _VP, _VP],
    "mfc_fill_ghosts": [_VP, _VP, _VP],
    "mfc_rhs": [_VP, _VP, _VP, _VP],
    "mfc_rhs_noalloc": [ctypes.POINTER(mfc_grid_desc), _VP, _VP, _VP, _VP],
    "mfc_max_wavespeed": [_VP, _VP, ctypes.POINTER(ctypes.c_double), _VP],
    "mfc_rk3_step": [_VP, _VP, ctypes.c_double, ctypes.c_double, _VP, _VP],
    "mfc_run": [_VP, _VP, ctypes.c_int, ctypes.c_double, ctypes.c_double, _VP],
    "mfc_time": [_VP, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double), _VP],
    "mfc_reset_time": [_VP, _VP],
    "mfc_check": [_VP, _VP],
    "mfc_set_kernel_timing": [_VP, ctypes.c_int],
    "mfc_kernel_time": [_VP, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)],
    "mfc_set_indicator": [_VP, ctypes.POINTER(ctypes.c_float), ctypes.c_double],
    "mfc_harvest": [_VP, _VP, _VP, _VP, _VP, _VP],
    "mfc_trainer_init": [ctypes.c_int64, ctypes.POINTER(_VP)],
    "mfc_trainer_free": [_VP],
    "mfc_trainer_set_params": [_VP, ctypes.POINTER(ctypes.c_float)],
    "mfc_trainer_get_params": [_VP, ctypes.POINTER(ctypes.c_float)],
    "mfc_trainer_grad": [_VP, _VP, _VP, _VP, ctypes.c_int64, _VP],
    "mfc_trainer_read_grad": [_VP, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float), _VP],
    "mfc_trainer_adam": [_VP, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float, _VP],
    "mfc_trainer_infer": [_VP, _VP, ctypes.c_int64, _VP, _VP],
    "mfc_batch_init": [ctypes.POINTER(mfc_grid_desc), ctypes.c_int, ctypes.POINTER(_VP)],
    "mfc_batch_free": [_VP],
    "mfc_batch_layout": [_VP, ctypes.c_int, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                         ctypes.POINTER(ctypes.c_int64)],
    "mfc_batch_cells": [_VP, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int)],
    "mfc_batch_step": [_VP, ctypes.POINTER(_VP), ctypes.c_double, _VP],
    "mfc_batch_run": [_VP, ctypes.POINTER(_VP), ctypes.c_int, ctypes.c_double, ctypes.c_int, _VP],
    "mfc_batch_autotune": [_VP, ctypes.POINTER(_VP), ctypes.c_int, ctypes.POINTER(mfc_batch_tune),
                           ctypes.POINTER(ctypes.c_double), _VP],
    "mfc_batch_set_tune": [_VP, ctypes.POINTER(mfc_batch_tune)],
    "mfc_batch_get_tune": [_VP, ctypes.POINTER(mfc_batch_tune)],
    "mfc_batch_set_timing": [_VP, ctypes.c_int],
    "mfc_batch_kernel_time": [_VP, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)],
    "mfc_batch_time": [_VP, ctypes.POINTER(ctypes.c_double), _VP],
    "mfc_batch_check": [_VP, _VP],
}


def header_symbols() -> list[str]:
    """Names of the functions include/mfc.h declares."""
    text = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(mfc_\w+)\s*\(", text, re.M)))


def lib():
    """Load libmfc.so (after torch, so that one HIP runtime serves both)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python __graft_entry__.py build` "
                               "(or paper_2305_09163_amd/build.py) first; there is no CPU fallback")
        import torch  # noqa: F401  (loads the HIP runtime the library then shares)
        L = ctypes.CDLL(LIB_PATH)
        for name, args in _SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = ctypes.c_int
        L.mfc_strerror.argtypes = [ctypes.c_int]
        L.mfc_strerror.restype = ctypes.c_char_p
        L.mfc_last_error_detail.argtypes = []
        L.mfc_last_error_detail.restype = ctypes.c_char_p
        _lib = L
    return _lib


def _check(status: int, call: str):
    if status != MFC_OK:
        L = lib()
        raise MfcError(status, call, f"{L.mfc_strerror(status).decode()}: {L.mfc_last_error_detail().decode()}")


def _stream(stream=None):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return _VP(stream.cuda_stream)


def _ptr(t):
    return _VP(t.data_ptr())


def make_desc(spec, precision: int = MFC_FP64, recon: int = MFC_RECON_WENO5,
              kernel: int = MFC_KERNEL_FUSED) -> mfc_grid_desc:
    """C descriptor from a GridSpec-like object (ndim, n, lo, hi, gamma, pi_inf, bc, weno_eps and,
    if present, model)."""
    d = mfc_grid_desc()
    d.ndim = spec.ndim
    for k in range(3):
        d.n[k] = spec.n[k]
        d.lo[k] = spec.lo[k]
        d.hi[k] = spec.hi[k]
    d.num_fluids = 2
    d.gamma[0], d.gamma[1] = spec.gamma
    d.pi_inf[0], d.pi_inf[1] = spec.pi_inf
    for f in range(6):
        d.bc[f] = spec.bc[f]
    d.precision = precision
    d.recon = recon
    d.weno_eps = spec.weno_eps
    d.kernel = kernel
    d.model = getattr(spec, "model", MFC_MODEL_ALLAIRE)
    d._keep = []   # face arrays must outlive the init call that copies them
    for k in range(3):
        f = spec.face_coords(k) if hasattr(spec, "face_coords") else None
        if f is not None:
            f = np.ascontiguousarray(f, dtype=np.float64)
            d._keep.append(f)
            d.faces[k] = f.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    return d


# ---------------------------------------------------------------------------
# Thin wrappers with the C names (status codes raised as MfcError)
# ---------------------------------------------------------------------------

def mfc_init_grid(desc: mfc_grid_desc) -> ctypes.c_void_p:
    h = _VP()
    _check(lib().mfc_init_grid(ctypes.byref(desc), ctypes.byref(h)), "mfc_init_grid")
    return h


def mfc_free_grid(h):
    _check(lib().mfc_free_grid(h), "mfc_free_grid")


def mfc_state_layout(h):
    nv, eb = ctypes.c_int64(), ctypes.c_int64()
    pad = (ctypes.c_int64 * 3)()
    _check(lib().mfc_state_layout(h, ctypes.byref(nv), pad, ctypes.byref(eb)), "mfc_state_layout")
    return nv.value, tuple(pad), eb.value


def mfc_prim_to_cons(h, w, q, stream=None):
    _check(lib().mfc_prim_to_cons(h, _ptr(w), _ptr(q), _stream(stream)), "mfc_prim_to_cons")


def mfc_cons_to_prim(h, q, w, stream=None):
    _check(lib().mfc_cons_to_prim(h, _ptr(q), _ptr(w), _stream(stream)), "mfc_cons_to_prim")


def mfc_fill_ghosts(h, q, stream=None):
    _check(lib().mfc_fill_ghosts(h, _ptr(q), _stream(stream)), "mfc_fill_ghosts")


def mfc_rhs(h, q, rhs, stream=None):
    _check(lib().mfc_rhs(h, _ptr(q), _ptr(rhs), _stream(stream)), "mfc_rhs")


def mfc_max_wavespeed(h, q, stream=None) -> float:
    s = ctypes.c_double()
    _check(lib().mfc_max_wavespeed(h, _ptr(q), ctypes.byref(s), _stream(stream)), "mfc_max_wavespeed")
    return s.value


def mfc_rk3_step(h, q, cfl: float = 0.0, dt: float = 0.0, dt_used=None, stream=None):
    """One SSP-RK3 step; dt_used: optional device float64 tensor that receives
    the step size taken."""
    _check(lib().mfc_rk3_step(h, _ptr(q), cfl, dt, _ptr(dt_used) if dt_used is not None else None,
                              _stream(stream)), "mfc_rk3_step")


def mfc_run(h, q, nsteps: int, cfl: float = 0.0, dt: float = 0.0, stream=None):
    _check(lib().mfc_run(h, _ptr(q), nsteps, cfl, dt, _stream(stream)), "mfc_run")


def mfc_rhs_noalloc(desc, q, rhs, flag, stream=None):
    """The right-hand side of mfc_rhs on the split kernels with no grid handle
    and no device allocation; `flag` is a device int32 tensor that the
    kernels set nonzero on a non-physical cell (the caller clears it)."""
    _check(lib().mfc_rhs_noalloc(ctypes.byref(desc), _ptr(q), _ptr(rhs), _ptr(flag), _stream(stream)),
           "mfc_rhs_noalloc")


def mfc_time(h, stream=None):
    t, dt = ctypes.c_double(), ctypes.c_double()
    _check(lib().mfc_time(h, ctypes.byref(t), ctypes.byref(dt), _stream(stream)), "mfc_time")
    return t.value, dt.value


def mfc_reset_time(h, stream=None):
    _check(lib().mfc_reset_time(h, _stream(stream)), "mfc_reset_time")


def mfc_check(h, stream=None):
    _check(lib().mfc_check(h, _stream(stream)), "mfc_check")


def mfc_set_kernel_timing(h, enable: bool, stride: int = 1):
    _check(lib().mfc_set_kernel_timing(h, int(stride) if enable else 0), "mfc_set_kernel_timing")


def mfc_kernel_time(h, slot: int = 0):
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(lib().mfc_kernel_time(h, slot, ctypes.byref(ms), ctypes.byref(n)), "mfc_kernel_time")
    return ms.value, n.value


# ---------------------------------------------------------------------------
# Convenience object
# ---------------------------------------------------------------------------

class Solver:
    """A grid handle plus torch-allocated state helpers."""

    def __init__(self, spec, precision: int = MFC_FP64, recon: int = MFC_RECON_WENO5,
                 kernel: int = MFC_KERNEL_FUSED):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible; the library runs on the GPU only")
        self.spec = spec
        self.desc = make_desc(spec, precision, recon, kernel)
        self.h = mfc_init_grid(self.desc)
        nv, pad, eb = mfc_state_layout(self.h)
        self.shape = (nv, pad[2], pad[1], pad[0])
        self.dtype = torch.float64 if eb == 8 else torch.float32

    def close(self):
        if self.h:
            mfc_free_grid(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def empty(self):
        import torch
        return torch.empty(self.shape, dtype=self.dtype, device="cuda")

    def state_from_prim(self, w_host):
        """Conservative device state from a host primitive array (converted on the GPU)."""
        import torch
        w = torch.as_tensor(w_host, dtype=self.dtype).to("cuda")
        q = self.empty()
        mfc_prim_to_cons(self.h, w, q)
        return q

    def upload(self, q_host):
        """Device copy of a host conservative state of this grid's padded
        layout, in the storage type (no conversion beyond that rounding)."""
        import torch
        if tuple(q_host.shape) != self.shape:
            raise ValueError(f"state shape {tuple(q_host.shape)} is not the grid's {self.shape}")
        return torch.as_tensor(q_host, dtype=self.dtype).to("cuda").contiguous()

    def fill_ghosts(self, q):
        mfc_fill_ghosts(self.h, q)

    def rhs(self, q, out=None):
        import torch
        if out is None:
            out = torch.zeros_like(q)
        mfc_rhs(self.h, q, out)
        return out

    def max_wavespeed(self, q):
        return mfc_max_wavespeed(self.h, q)

    def step(self, q, cfl=0.0, dt=0.0, dt_used=None):
        mfc_rk3_step(self.h, q, cfl, dt, dt_used)

    def run(self, q, nsteps, cfl=0.0, dt=0.0):
        mfc_run(self.h, q, nsteps, cfl, dt)

    def time(self):
        return mfc_time(self.h)

    def check(self):
        mfc_check(self.h)

    def set_indicator(self, params, tau):
        mfc_set_indicator(self.h, params, tau)

    def harvest(self, q):
        """(features [ndim*cells, 16] int16 bf16 bits, labels uint8, max deviation float64), on the device."""
        import torch
        n = self.spec.cells * self.spec.ndim
        X = torch.empty((n, 16), dtype=torch.int16, device="cuda")
        Y = torch.empty(n, dtype=torch.uint8, device="cuda")
        D = torch.empty(n, dtype=torch.float64, device="cuda")
        mfc_harvest(self.h, q, X, Y, D)
        return X, Y, D


# ---------------------------------------------------------------------------
# Learned indicator
# ---------------------------------------------------------------------------

NPARAM = 1601


def _fptr(a):
    import numpy as np
    assert a.dtype == np.float32 and a.flags["C_CONTIGUOUS"] and a.size == NPARAM
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def mfc_set_indicator(h, params, tau: float):
    import numpy as np
    p = np.ascontiguousarray(params, dtype=np.float32)
    _check(lib().mfc_set_indicator(h, _fptr(p), tau), "mfc_set_indicator")


def mfc_harvest(h, q, features, labels, maxdev=None, stream=None):
    _check(lib().mfc_harvest(h, _ptr(q), _ptr(features), _ptr(labels), _ptr(maxdev) if maxdev is not None else None,
                             _stream(stream)), "mfc_harvest")


class Trainer:
    """FP32 master weights + Adam on the device; gradients from the library's
    bf16 matrix-core kernels."""

    def __init__(self, max_batch: int):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible; the library runs on the GPU only")
        self.t = _VP()
        _check(lib().mfc_trainer_init(max_batch, ctypes.byref(self.t)), "mfc_trainer_init")
        self.max_batch = max_batch

    def close(self):
        if self.t:
            _check(lib().mfc_trainer_free(self.t), "mfc_trainer_free")
            self.t = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_params(self, flat):
        import numpy as np
        p = np.ascontiguousarray(flat, dtype=np.float32)
        _check(lib().mfc_trainer_set_params(self.t, _fptr(p)), "mfc_trainer_set_params")

    def params(self):
        import numpy as np
        p = np.empty(NPARAM, dtype=np.float32)
        _check(lib().mfc_trainer_get_params(self.t, _fptr(p)), "mfc_trainer_get_params")
        return p

    def grad(self, X, Y, index=None, batch=None):
        batch = (index.numel() if index is not None else X.shape[0]) if batch is None else batch
        _check(lib().mfc_trainer_grad(self.t, _ptr(X), _ptr(Y), _ptr(index) if index is not None else None, batch,
                                      _stream(None)), "mfc_trainer_grad")

    def read_grad(self):
        import numpy as np
        g = np.empty(NPARAM, dtype=np.float32)
        loss = ctypes.c_float()
        _check(lib().mfc_trainer_read_grad(self.t, _fptr(g), ctypes.byref(loss), _stream(None)),
               "mfc_trainer_read_grad")
        return g, loss.value

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        _check(lib().mfc_trainer_adam(self.t, lr, beta1, beta2, eps, _stream(None)), "mfc_trainer_adam")

    def infer(self, X):
        import torch
        prob = torch.empty(X.shape[0], dtype=torch.float32, device="cuda")
        _check(lib().mfc_trainer_infer(self.t, _ptr(X), X.shape[0], _ptr(prob), _stream(None)), "mfc_trainer_infer")
        return prob


# ---------------------------------------------------------------------------
# Batched ensembles of 2D runs
# ---------------------------------------------------------------------------

def _ptr_array(qs):
    return (_VP * len(qs))(*[q.data_ptr() for q in qs])


def mfc_batch_init(descs) -> ctypes.c_void_p:
    arr = (mfc_grid_desc * len(descs))(*descs)
    h = _VP()
    _check(lib().mfc_batch_init(arr, len(descs), ctypes.byref(h)), "mfc_batch_init")
    return h


def mfc_batch_free(b):
    _check(lib().mfc_batch_free(b), "mfc_batch_free")


def mfc_batch_layout(b, run: int):
    nv, eb = ctypes.c_int64(), ctypes.c_int64()
    pad = (ctypes.c_int64 * 3)()
    _check(lib().mfc_batch_layout(b, run, ctypes.byref(nv), pad, ctypes.byref(eb)), "mfc_batch_layout")
    return nv.value, tuple(pad), eb.value


def mfc_batch_cells(b):
    c, n = ctypes.c_int64(), ctypes.c_int()
    _check(lib().mfc_batch_cells(b, ctypes.byref(c), ctypes.byref(n)), "mfc_batch_cells")
    return c.value, n.value


def mfc_batch_step(b, qs, cfl: float, stream=None):
    _check(lib().mfc_batch_step(b, _ptr_array(qs), cfl, _stream(stream)), "mfc_batch_step")


def mfc_batch_run(b, qs, nsteps: int, cfl: float, use_graph: bool = True, stream=None):
    _check(lib().mfc_batch_run(b, _ptr_array(qs), nsteps, cfl, int(use_graph), _stream(stream)), "mfc_batch_run")


def mfc_batch_autotune(b, qs, reps: int = 5, stream=None):
    best = mfc_batch_tune()
    table = (ctypes.c_double * 18)()
    _check(lib().mfc_batch_autotune(b, _ptr_array(qs), reps, ctypes.byref(best), table, _stream(stream)),
           "mfc_batch_autotune")
    return (best.shape, best.groups, best.xcd), list(table)


def mfc_batch_set_tune(b, shape: int, groups: int, xcd: int):
    t = mfc_batch_tune(shape, groups, xcd)
    _check(lib().mfc_batch_set_tune(b, ctypes.byref(t)), "mfc_batch_set_tune")


def mfc_batch_get_tune(b):
    t = mfc_batch_tune()
    _check(lib().mfc_batch_get_tune(b, ctypes.byref(t)), "mfc_batch_get_tune")
    return t.shape, t.groups, t.xcd


def mfc_batch_set_timing(b, enable: bool):
    _check(lib().mfc_batch_set_timing(b, int(enable)), "mfc_batch_set_timing")


def mfc_batch_kernel_time(b):
    ms, n = ctypes.c_double(), ctypes.c_int64()
    _check(lib().mfc_batch_kernel_time(b, ctypes.byref(ms), ctypes.byref(n)), "mfc_batch_kernel_time")
    return ms.value, n.value


def mfc_batch_time(b, nrun: int, stream=None):
    t = (ctypes.c_double * nrun)()
    _check(lib().mfc_batch_time(b, t, _stream(stream)), "mfc_batch_time")
    return list(t)


def mfc_batch_check(b, stream=None):
    _check(lib().mfc_batch_check(b, _stream(stream)), "mfc_batch_check")


class Batch:
    """A batch handle for a list of 2D GridSpecs plus torch state helpers."""

    def __init__(self, specs, precision: int = MFC_FP32_MIXED):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no HIP device visible; the library runs on the GPU only")
        self.specs = list(specs)
        self.b = mfc_batch_init([make_desc(s, precision) for s in self.specs])
        self.cells, self.nrun = mfc_batch_cells(self.b)
        self.shapes = []
        for r in range(self.nrun):
            nv, pad, eb = mfc_batch_layout(self.b, r)
            self.shapes.append((nv, pad[2], pad[1], pad[0]))
        self.dtype = torch.float64 if eb == 8 else torch.float32
        self.precision = precision

    def close(self):
        if self.b:
            mfc_batch_free(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def states_from_prim(self, ws):
        """Device states from host primitive arrays, converted on the GPU by
        single-grid handles of the same runs."""
        qs = []
        for spec, w in zip(self.specs, ws):
            s = Solver(spec, precision=self.precision)
            qs.append(s.state_from_prim(w))
            s.close()
        return qs

    def upload(self, qs_host):
        """Device copies of host conservative states, one per run, each in
        its run's padded layout and the storage type."""
        qs = []
        for spec, qh in zip(self.specs, qs_host):
            s = Solver(spec, precision=self.precision)
            qs.append(s.upload(qh))
            s.close()
        return qs

    def step(self, qs, cfl):
        mfc_batch_step(self.b, qs, cfl)

    def run(self, qs, nsteps, cfl, use_graph=True):
        mfc_batch_run(self.b, qs, nsteps, cfl, use_graph)

    def autotune(self, qs, reps=5):
        return mfc_batch_autotune(self.b, qs, reps)

    def set_tune(self, shape, groups, xcd):
        mfc_batch_set_tune(self.b, shape, groups, xcd)

    def tune(self):
        return mfc_batch_get_tune(self.b)

    def time(self):
        return mfc_batch_time(self.b, self.nrun)

    def check(self):
        mfc_batch_check(self.b)
