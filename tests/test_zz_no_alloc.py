"""mfc_rhs_noalloc (the right-hand side with no grid handle and no device
allocation; its scratch is a fixed device array) against mfc_rhs on the split
kernels through the C ABI: the same kernels on the same input give the same
bits.  Two calls in a row, the second on a smaller grid, so that the second
reads scratch that the first left behind."""
import sys

import numpy as np
import pytest

import oracle
from paper_2305_09163_amd import mfc
from paper_2305_09163_amd import workloads as W

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, file=sys.stderr, flush=True)


CASES = [
    # (first grid, second grid, precision, reconstruction)
    ((37, 29, 23), (24, 20, 17), mfc.MFC_FP64, mfc.MFC_RECON_WENO5),
    ((44, 33, 35), (19, 26, 9), mfc.MFC_FP32_MIXED, mfc.MFC_RECON_WENO5),
    ((30, 22, 41), (13, 11, 12), mfc.MFC_FP64, mfc.MFC_RECON_WENO3),
]


@pytest.mark.parametrize("first,second,precision,recon", CASES)
def test_noalloc_rhs_equals_mfc_rhs(first, second, precision, recon):
    import torch
    assert torch.cuda.is_available()
    for n in (first, second):
        spec, w = W.bubble_collapse_3d(n=n)
        say(f"[noalloc] grid {n} precision {precision} recon {recon}")
        s = mfc.Solver(spec, precision=precision, recon=recon, kernel=mfc.MFC_KERNEL_SPLIT)
        q = s.upload(oracle.prim_to_cons_field(spec, w))
        ref = torch.zeros_like(q)
        mfc.mfc_rhs(s.h, q, ref)
        s.check()
        got = torch.full_like(q, float("nan"))   # ghost entries must stay as they were
        flag = torch.zeros(1, dtype=torch.int32, device="cuda")
        desc = mfc.make_desc(spec, precision, recon, mfc.MFC_KERNEL_SPLIT)
        mfc.mfc_rhs_noalloc(desc, q, got, flag)
        torch.cuda.synchronize()
        assert int(flag.item()) == 0
        I = (slice(None),) + spec.interior[1:]
        a, b = got.cpu().numpy(), ref.cpu().numpy()
        assert np.array_equal(a[I], b[I]), float(np.nanmax(np.abs(a[I] - b[I])))
        ghost = np.ones(a.shape, dtype=bool)
        ghost[I] = False
        assert np.isnan(a[ghost]).all()


def test_noalloc_rhs_flags_nonphysical():
    """A cell with negative density sets the caller's flag (the result is
    then undefined) and an uncleared flag stays set."""
    import torch
    spec, w = W.bubble_collapse_3d(n=(20, 18, 16))
    q0 = oracle.prim_to_cons_field(spec, w)
    q0[0, 10, 10, 10] = -1.0
    q0[1, 10, 10, 10] = -1.0
    q = torch.as_tensor(q0).cuda()
    out = torch.zeros_like(q)
    flag = torch.zeros(1, dtype=torch.int32, device="cuda")
    desc = mfc.make_desc(spec, mfc.MFC_FP64, mfc.MFC_RECON_WENO5, mfc.MFC_KERNEL_SPLIT)
    mfc.mfc_rhs_noalloc(desc, q, out, flag)
    torch.cuda.synchronize()
    assert int(flag.item()) != 0
