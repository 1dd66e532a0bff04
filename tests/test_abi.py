"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/mfc.h declares, and rejects invalid arguments with
the documented status codes before touching the device."""
import ctypes
import os

import pytest

from paper_2305_09163_amd import mfc
from paper_2305_09163_amd import workloads as W


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(mfc.LIB_PATH):
        pytest.fail("libmfc.so is not built (run __graft_entry__.build())")
    return mfc.lib()


def test_exports_every_declared_symbol(L):
    names = mfc.header_symbols()
    assert "mfc_rhs" in names and "mfc_rk3_step" in names and len(names) >= 15
    for name in names:
        assert hasattr(L, name), name


def test_strerror(L):
    for code in (mfc.MFC_OK, mfc.MFC_E_ARG, mfc.MFC_E_NOMEM, mfc.MFC_E_HIP, mfc.MFC_E_NONPHYSICAL,
                 mfc.MFC_E_UNSUPPORTED):
        assert len(L.mfc_strerror(code)) > 0
    assert L.mfc_strerror(12345) == b"unknown status"


def desc(**kw):
    spec = W.GridSpec(ndim=3, n=(8, 8, 8))
    d = mfc.make_desc(spec, kernel=mfc.MFC_KERNEL_STAGED)
    for k, v in kw.items():
        if isinstance(v, (list, tuple)):
            arr = getattr(d, k)
            for i, x in enumerate(v):
                arr[i] = x
        else:
            setattr(d, k, v)
    return d


@pytest.mark.parametrize("kw,code", [
    (dict(ndim=0), mfc.MFC_E_ARG),
    (dict(ndim=4), mfc.MFC_E_ARG),
    (dict(n=(2, 8, 8)), mfc.MFC_E_ARG),
    (dict(num_fluids=3), mfc.MFC_E_UNSUPPORTED),
    (dict(gamma=(1.0, 1.4)), mfc.MFC_E_ARG),
    (dict(pi_inf=(-1.0, 0.0)), mfc.MFC_E_ARG),
    (dict(hi=(0.0, 1.0, 1.0)), mfc.MFC_E_ARG),
    (dict(bc=(1, 0, 0, 0, 0, 0)), mfc.MFC_E_ARG),
    (dict(bc=(7, 7, 0, 0, 0, 0)), mfc.MFC_E_ARG),
    (dict(weno_eps=0.0), mfc.MFC_E_ARG),
    (dict(precision=9), mfc.MFC_E_ARG),
    (dict(kernel=9), mfc.MFC_E_ARG),
    (dict(model=2), mfc.MFC_E_ARG),
    (dict(recon=9), mfc.MFC_E_ARG),
])
def test_init_rejects_invalid_descriptors(L, kw, code):
    h = ctypes.c_void_p(123)
    st = L.mfc_init_grid(ctypes.byref(desc(**kw)), ctypes.byref(h))
    assert st == code
    assert h.value is None
    assert len(L.mfc_last_error_detail()) > 0


def test_null_arguments(L):
    assert L.mfc_init_grid(None, None) == mfc.MFC_E_ARG
    h = ctypes.c_void_p()
    assert L.mfc_init_grid(None, ctypes.byref(h)) == mfc.MFC_E_ARG
    for name in ("mfc_fill_ghosts", "mfc_check", "mfc_reset_time"):
        f = getattr(L, name)
        args = [None] * (len(f.argtypes))
        assert f(*args) == mfc.MFC_E_ARG, name
    assert L.mfc_rhs(None, None, None, None) == mfc.MFC_E_ARG
    assert L.mfc_rk3_step(None, None, 0.3, 0.0, None, None) == mfc.MFC_E_ARG
    assert L.mfc_free_grid(None) == mfc.MFC_OK


def batch_descs(count=3, **kw):
    out = []
    for r in range(count):
        spec = W.GridSpec(ndim=2, n=(16 + 8 * r, 24))
        d = mfc.make_desc(spec, precision=mfc.MFC_FP32_MIXED)
        out.append(d)
    for k, v in kw.items():
        d = out[-1]
        if isinstance(v, (list, tuple)):
            arr = getattr(d, k)
            for i, x in enumerate(v):
                arr[i] = x
        else:
            setattr(d, k, v)
    return (mfc.mfc_grid_desc * count)(*out)


@pytest.mark.parametrize("kw,code", [
    (dict(ndim=3), mfc.MFC_E_UNSUPPORTED),
    (dict(ndim=1), mfc.MFC_E_UNSUPPORTED),
    (dict(precision=mfc.MFC_FP64), mfc.MFC_E_ARG),   # mixed precisions in one batch
    (dict(num_fluids=3), mfc.MFC_E_UNSUPPORTED),
    (dict(recon=mfc.MFC_RECON_LEARNED), mfc.MFC_E_UNSUPPORTED),
    (dict(model=-1), mfc.MFC_E_ARG),
    (dict(recon=mfc.MFC_RECON_WENO3), mfc.MFC_E_UNSUPPORTED),
    (dict(n=(2, 24, 1)), mfc.MFC_E_ARG),
    (dict(n=(40000, 24, 1)), mfc.MFC_E_ARG),
    (dict(gamma=(0.9, 1.4)), mfc.MFC_E_ARG),
    (dict(bc=(1, 0, 0, 0, 0, 0)), mfc.MFC_E_ARG),
    (dict(hi=(0.0, 1.0, 1.0)), mfc.MFC_E_ARG),
    (dict(weno_eps=-1.0), mfc.MFC_E_ARG),
])
def test_batch_init_rejects_invalid_descriptors(L, kw, code):
    b = ctypes.c_void_p(123)
    assert L.mfc_batch_init(batch_descs(**kw), 3, ctypes.byref(b)) == code
    assert b.value is None


def test_batch_null_arguments(L):
    b = ctypes.c_void_p()
    assert L.mfc_batch_init(None, 3, ctypes.byref(b)) == mfc.MFC_E_ARG
    assert L.mfc_batch_init(batch_descs(), 0, ctypes.byref(b)) == mfc.MFC_E_ARG
    assert L.mfc_batch_init(batch_descs(), 3, None) == mfc.MFC_E_ARG
    assert L.mfc_batch_step(None, None, 0.3, None) == mfc.MFC_E_ARG
    assert L.mfc_batch_run(None, None, 1, 0.3, 1, None) == mfc.MFC_E_ARG
    assert L.mfc_batch_autotune(None, None, 1, None, None, None) == mfc.MFC_E_ARG
    assert L.mfc_batch_set_tune(None, None) == mfc.MFC_E_ARG
    assert L.mfc_batch_check(None, None) == mfc.MFC_E_ARG
    assert L.mfc_batch_time(None, None, None) == mfc.MFC_E_ARG
    assert L.mfc_batch_free(None) == mfc.MFC_OK


def test_learned_null_arguments(L):
    assert L.mfc_set_indicator(None, None, 0.5) == mfc.MFC_E_ARG
    assert L.mfc_harvest(None, None, None, None, None, None) == mfc.MFC_E_ARG
    assert L.mfc_trainer_init(0, ctypes.byref(ctypes.c_void_p())) == mfc.MFC_E_ARG
    assert L.mfc_trainer_init(16, None) == mfc.MFC_E_ARG
    assert L.mfc_trainer_grad(None, None, None, None, 1, None) == mfc.MFC_E_ARG
    assert L.mfc_trainer_read_grad(None, None, None, None) == mfc.MFC_E_ARG
    assert L.mfc_trainer_adam(None, 1e-3, 0.9, 0.999, 1e-8, None) == mfc.MFC_E_ARG
    assert L.mfc_trainer_infer(None, None, 1, None, None) == mfc.MFC_E_ARG
    assert L.mfc_trainer_set_params(None, None) == mfc.MFC_E_ARG
    assert L.mfc_trainer_free(None) == mfc.MFC_OK


def test_learned_recon_rejected_for_staged(L):
    h = ctypes.c_void_p(123)
    d = desc(recon=mfc.MFC_RECON_LEARNED)      # desc() builds a staged-kernel descriptor
    assert L.mfc_init_grid(ctypes.byref(d), ctypes.byref(h)) == mfc.MFC_E_UNSUPPORTED


@pytest.mark.parametrize("kernel,recon,faces,code", [
    (mfc.MFC_KERNEL_SPLIT, mfc.MFC_RECON_WENO3, "tanh", mfc.MFC_E_UNSUPPORTED),
    (mfc.MFC_KERNEL_SPLIT, mfc.MFC_RECON_LEARNED, "tanh", mfc.MFC_E_UNSUPPORTED),
    (mfc.MFC_KERNEL_STAGED, mfc.MFC_RECON_WENO5, "tanh", mfc.MFC_E_UNSUPPORTED),
    (mfc.MFC_KERNEL_FUSED, mfc.MFC_RECON_WENO3, "tanh", mfc.MFC_E_UNSUPPORTED),
    (mfc.MFC_KERNEL_FUSED, mfc.MFC_RECON_LEARNED, "tanh", mfc.MFC_E_UNSUPPORTED),
    (mfc.MFC_KERNEL_FUSED, mfc.MFC_RECON_WENO5, "unsorted", mfc.MFC_E_ARG),
    (mfc.MFC_KERNEL_FUSED, mfc.MFC_RECON_WENO5, "nan", mfc.MFC_E_ARG),
])
def test_init_rejects_unsupported_non_uniform_grids(L, kernel, recon, faces, code):
    import dataclasses
    spec, _ = W.bubble_collapse_3d(n=(8, 8, 8))
    f = W.tanh_faces(8, depth=0.5)
    if faces == "unsorted":
        f = f.copy()
        f[3], f[4] = f[4], f[3]
    elif faces == "nan":
        f = f.copy()
        f[2] = float("nan")
    spec = dataclasses.replace(spec, faces=(f, None, None))
    d = mfc.make_desc(spec, kernel=kernel, recon=recon)
    h = ctypes.c_void_p(123)
    assert L.mfc_init_grid(ctypes.byref(d), ctypes.byref(h)) == code
    assert h.value is None


@pytest.mark.parametrize("kw,code", [
    (dict(bc=(2, 2, 0, 0, 0, 0), model=mfc.MFC_MODEL_KAPILA), mfc.MFC_E_UNSUPPORTED),
    (dict(bc=(0, 0, 0, 0, 2, 0), kernel=mfc.MFC_KERNEL_FUSED, recon=mfc.MFC_RECON_LEARNED), mfc.MFC_E_UNSUPPORTED),
    (dict(bc=(2, 1, 0, 0, 0, 0)), mfc.MFC_E_ARG),       # periodic on one face only
    (dict(bc=(3, 0, 0, 0, 0, 0)), mfc.MFC_E_ARG),
])
def test_init_rejects_unsupported_characteristic_faces(L, kw, code):
    h = ctypes.c_void_p(123)
    assert L.mfc_init_grid(ctypes.byref(desc(**kw)), ctypes.byref(h)) == code
    assert h.value is None


def test_characteristic_faces_on_non_uniform_cells(L):
    """Characteristic faces combine with non-uniform cells on the fused and
    split kernels (validation passes: without a device the call fails later,
    at the device query), not on the staged kernel."""
    import dataclasses
    spec, _ = W.bubble_collapse_3d(n=(8, 8, 8))
    spec = dataclasses.replace(spec, faces=(None, W.tanh_faces(8, depth=0.5), None), bc=(2, 2, 0, 0, 0, 0))
    for kernel, ok in ((mfc.MFC_KERNEL_FUSED, True), (mfc.MFC_KERNEL_SPLIT, True), (mfc.MFC_KERNEL_STAGED, False)):
        d = mfc.make_desc(spec, kernel=kernel)
        h = ctypes.c_void_p(123)
        st = L.mfc_init_grid(ctypes.byref(d), ctypes.byref(h))
        assert (st != mfc.MFC_E_UNSUPPORTED) if ok else (st == mfc.MFC_E_UNSUPPORTED), (kernel, st)
        if st != mfc.MFC_OK:
            assert h.value is None
        else:
            L.mfc_free_grid(h)


def test_batch_characteristic_faces(L):
    """Batched runs take characteristic faces with the Allaire model
    (validation passes: without a device the call fails later), not with
    the Kapila model, and a periodic face still needs its partner."""
    b = ctypes.c_void_p(123)
    st = L.mfc_batch_init(batch_descs(bc=(2, 2, 0, 0, 0, 0)), 3, ctypes.byref(b))
    assert st not in (mfc.MFC_E_ARG, mfc.MFC_E_UNSUPPORTED), st
    if st == mfc.MFC_OK:
        L.mfc_batch_free(b)
    b = ctypes.c_void_p(123)
    assert L.mfc_batch_init(batch_descs(bc=(2, 2, 0, 0, 0, 0), model=mfc.MFC_MODEL_KAPILA), 3,
                            ctypes.byref(b)) == mfc.MFC_E_UNSUPPORTED
    assert b.value is None
    assert L.mfc_batch_init(batch_descs(bc=(2, 1, 0, 0, 0, 0)), 3, ctypes.byref(b)) == mfc.MFC_E_ARG
    assert b.value is None


def test_noalloc_rhs_rejects_on_the_host(L):
    """mfc_rhs_noalloc checks its arguments before any device call: null
    pointers, descriptors mfc_init_grid would reject, configurations outside
    the 3D split kernels, and grids whose x+y part exceeds its 64 MiB
    scratch (nvar x padded cells x element size)."""
    fake = ctypes.c_void_p(256)   # never dereferenced: every case fails first

    def call(d, q=fake, r=ctypes.c_void_p(512), f=ctypes.c_void_p(768)):
        return L.mfc_rhs_noalloc(ctypes.byref(d) if d is not None else None, q, r, f, None)

    def d3(n, **kw):
        d = mfc.make_desc(W.GridSpec(ndim=3, n=n), kernel=mfc.MFC_KERNEL_SPLIT)
        for k, v in kw.items():
            setattr(d, k, v)
        return d

    assert call(None) == mfc.MFC_E_ARG
    assert call(d3((8, 8, 8)), q=None) == mfc.MFC_E_ARG
    assert call(d3((8, 8, 8)), f=None) == mfc.MFC_E_ARG
    assert call(d3((8, 8, 8)), q=fake, r=fake) == mfc.MFC_E_ARG            # q and rhs alias
    assert call(desc(n=(2, 8, 8))) == mfc.MFC_E_ARG                         # what mfc_init_grid rejects
    d2 = mfc.make_desc(W.GridSpec(ndim=2, n=(16, 16)), kernel=mfc.MFC_KERNEL_FUSED)
    assert call(d2) == mfc.MFC_E_UNSUPPORTED                                # split kernels are 3D
    assert call(d3((8, 8, 8), recon=mfc.MFC_RECON_LEARNED)) == mfc.MFC_E_UNSUPPORTED
    dc = d3((8, 8, 8))
    dc.bc[0] = dc.bc[1] = mfc.MFC_BC_CHARACTERISTIC
    assert call(dc) == mfc.MFC_E_UNSUPPORTED
    # 7 x 107^3 x 8 B = 68.6 MB > 64 MiB in FP64; the same grid fits in FP32
    assert call(d3((101, 101, 101))) == mfc.MFC_E_ARG
    assert b"64 MiB" in L.mfc_last_error_detail()
