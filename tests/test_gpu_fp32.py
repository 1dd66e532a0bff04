"""FP32 storage form: float state, reconstruction and Riemann solve, with the
mixture pressure recovery and the HLLC contact speed in FP64.  Its error is
measured against the FP64 oracle on the same seeded inputs; the gate on
the bubble workload is the relative L1 density error <= 1e-4."""
import sys

import numpy as np
import pytest

import oracle
from parity_util import acoustic_floor, rel_l1, rel_linf
from paper_2305_09163_amd import mfc
from paper_2305_09163_amd import workloads as W

pytestmark = pytest.mark.gpu

KERNELS = {"fused": mfc.MFC_KERNEL_FUSED, "split": mfc.MFC_KERNEL_SPLIT}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def rho_l1(a, b, spec):
    I = spec.interior[1:]
    ra, rb = (a[0] + a[1])[I], (b[0] + b[1])[I]
    return np.abs(ra - rb).sum() / np.abs(rb).sum()


CASES = {
    "bubble_3d_37x21x19": (lambda: W.bubble_collapse_3d(n=(37, 21, 19)), ["fused", "split"]),
    "cloud_3d_40": (lambda: W.bubble_cloud_3d(n=40), ["fused", "split"]),
    "droplet_2d_45": (lambda: W.droplet_shock_2d(45, W.SEED + 11), ["fused"]),
    "shock_tube_400": (lambda: W.shock_tube_1d(400), ["fused"]),
}


@pytest.mark.parametrize("name,kernel", [(n, k) for n, (_, ks) in CASES.items() for k in ks])
def test_fp32_one_step_error(name, kernel):
    spec, w = CASES[name][0]()
    say(f"[fp32 1 step] {name} kernel={kernel}")
    s = mfc.Solver(spec, precision=mfc.MFC_FP32_MIXED, kernel=KERNELS[kernel])
    q = s.state_from_prim(w)
    s.step(q, cfl=0.3)
    s.check()
    qi = oracle.prim_to_cons_field(spec, w)
    qo, _, st = oracle.run(spec, qi, 1, cfl=0.3)
    assert st == oracle.OK
    got = host(q)
    fl = acoustic_floor(spec, qi)
    linf = rel_linf(got, qo, spec, floor_mom=fl)
    l1 = rel_l1(got, qo, spec, floor_mom=fl)
    say(f"    rel Linf {linf}\n    rel L1 {l1}\n    rho L1 {rho_l1(got, qo, spec):.3e}")
    assert rho_l1(got, qo, spec) <= 1e-6
    assert linf.max() <= 2e-4, linf
    assert l1.max() <= 2e-5, l1


@pytest.mark.parametrize("kernel", sorted(KERNELS))
def test_fp32_bubble_density_error_after_50_steps(kernel):
    """The bubble-collapse recipe at 48^3, 50 steps at CFL 0.3: relative L1
    density error against the FP64 oracle within the 1e-4 gate."""
    spec, w = W.bubble_collapse_3d(n=48)
    say(f"[fp32 50 steps] bubble_3d_48 kernel={kernel}")
    s = mfc.Solver(spec, precision=mfc.MFC_FP32_MIXED, kernel=KERNELS[kernel])
    q = s.state_from_prim(w)
    s.run(q, 50, cfl=0.3)
    s.check()
    qo, _, st = oracle.run(spec, oracle.prim_to_cons_field(spec, w), 50, cfl=0.3)
    assert st == oracle.OK
    err = rho_l1(host(q), qo, spec)
    fl = acoustic_floor(spec, oracle.prim_to_cons_field(spec, w))
    say(f"    rho L1 {err:.3e}; per-variable rel L1 {rel_l1(host(q), qo, spec, floor_mom=fl)}")
    assert err <= 1e-4


def test_fp32_bubble_cloud_64_after_50_steps():
    """The bubble-cloud recipe (50 air bubbles in water, a 1e7 Pa slab entering
    from x = 0) rebuilt at 64^3 from the same seeds and physical radii: 50
    steps at CFL 0.3 of the FP32 form (split path) against the FP64 oracle,
    relative L1 density error within the 1e-4 gate."""
    spec, w = W.bubble_cloud_3d(n=64)
    say("[fp32 50 steps] bubble_cloud_3d_64 kernel=split")
    s = mfc.Solver(spec, precision=mfc.MFC_FP32_MIXED, kernel=mfc.MFC_KERNEL_SPLIT)
    q = s.state_from_prim(w)
    s.run(q, 50, cfl=0.3)
    s.check()
    t_gpu, _ = s.time()
    qo, t_ora, st = oracle.run(spec, oracle.prim_to_cons_field(spec, w), 50, cfl=0.3)
    assert st == oracle.OK
    err = rho_l1(host(q), qo, spec)
    say(f"    rho L1 {err:.3e}; simulated time GPU {t_gpu:.6e} s, oracle {t_ora:.6e} s")
    assert abs(t_gpu - t_ora) <= 1e-5 * t_ora
    assert err <= 1e-4


def test_fp32_fused_and_split_agree():
    spec, w = W.bubble_collapse_3d(n=(37, 21, 19))
    outs = []
    for k in ("fused", "split"):
        s = mfc.Solver(spec, precision=mfc.MFC_FP32_MIXED, kernel=KERNELS[k])
        q = s.state_from_prim(w)
        s.run(q, 3, cfl=0.3)
        outs.append(host(q))
    err = rel_linf(outs[0], outs[1], spec, floor_mom=acoustic_floor(spec, oracle.prim_to_cons_field(spec, w)))
    assert err.max() <= 1e-5, err


def test_fp32_layout_and_dtype():
    spec, _ = W.bubble_collapse_3d(n=(19, 17, 16))
    s = mfc.Solver(spec, precision=mfc.MFC_FP32_MIXED)
    nv, pad, eb = mfc.mfc_state_layout(s.h)
    assert eb == 4 and nv == 7 and pad == (25, 23, 22)
    import torch
    assert s.empty().dtype == torch.float32
