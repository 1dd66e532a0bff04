"""Non-uniform (tanh-stretched) cells on the GPU (fused kernel; split
kernels in 3D) against the oracle's non-uniform scheme: right-hand side and
one step on 1D/2D/3D stretched grids for WENO5 and first order, multi-step
runs, the CFL step size, the FP32 form's error, and the split path's reading
of boundary neighbours without ghost cells."""
import dataclasses
import sys

import numpy as np
import pytest

import oracle
from parity_util import acoustic_floor, rel_l1, rel_linf, rhs_err, rounding_spread, run_parity, step_bar
from paper_2305_09163_amd import mfc
from paper_2305_09163_amd import workloads as W

pytestmark = pytest.mark.gpu
RECON = {"weno5": (mfc.MFC_RECON_WENO5, oracle.RECON_WENO5), "first": (mfc.MFC_RECON_FIRST_ORDER, oracle.RECON_FIRST)}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def with_faces(sw, faces):
    spec, w = sw
    return dataclasses.replace(spec, faces=faces), w


CASES = {
    "sine_1d_48": lambda: W.sine_advection_1d(48, stretch=0.5),
    "tube_1d_200": lambda: with_faces(W.shock_tube_1d(200), (W.tanh_faces(200, centre=0.7, depth=0.5), None, None)),
    "droplet_2d_40x33": lambda: with_faces(W.droplet_shock_2d((40, 33), W.SEED + 11),
                                           (W.tanh_faces(40, centre=0.4, depth=0.5), W.tanh_faces(33, depth=0.3), None)),
    "bubble_3d_17x15x17": lambda: W.bubble_collapse_3d(n=(17, 15, 17), stretch=0.6),
    "bubble_3d_x_only": lambda: with_faces(W.bubble_collapse_3d(n=(19, 16, 14)), (W.tanh_faces(19, depth=0.6), None, None)),
    # several x+y tiles and z chunks in every direction, ragged in x and y
    "bubble_3d_66x53x64": lambda: W.bubble_collapse_3d(n=(66, 53, 64), stretch=0.6),
}
KERNELS = {"fused": mfc.MFC_KERNEL_FUSED, "split": mfc.MFC_KERNEL_SPLIT}
PAIRS = [(name, r, k) for name in CASES for r in sorted(RECON) for k in sorted(KERNELS)
         if k == "fused" or CASES[name]()[0].ndim == 3]


@pytest.mark.parametrize("name,recon,kernel", PAIRS)
def test_rhs_and_step(name, recon, kernel):
    spec, w = CASES[name]()
    rg, ro_kind = RECON[recon]
    say(f"[stretched {recon} {kernel}] {name}")
    s = mfc.Solver(spec, kernel=KERNELS[kernel], recon=rg)
    q = s.upload(oracle.prim_to_cons_field(spec, w))
    s.fill_ghosts(q)
    r = s.rhs(q).cpu().numpy()
    s.check()
    qo = oracle.fill_ghosts(spec, oracle.prim_to_cons_field(spec, w))
    ro, st = oracle.rhs(spec, qo, recon=ro_kind)
    assert st == oracle.OK
    err = rhs_err(r, ro, qo, spec)
    q1 = s.upload(oracle.prim_to_cons_field(spec, w))
    s.step(q1, cfl=0.3)
    t, _ = s.time()
    s.check()
    qn, to, st = oracle.run(spec, oracle.prim_to_cons_field(spec, w), 1, cfl=0.3, recon=ro_kind)
    assert st == oracle.OK
    assert t == pytest.approx(to, rel=1e-12)
    e1 = rel_linf(q1.cpu().numpy(), qn, spec)
    say(f"    rhs err {err.max():.2e}, one-step rel Linf {e1.max():.2e}")
    bar = step_bar(rounding_spread(spec, oracle.prim_to_cons_field(spec, w), 1, cfl=0.3, recon=ro_kind))
    assert err.max() <= 1e-12 and (e1 <= bar).all(), (e1, bar)


def test_sine_200_steps():
    spec, w = W.sine_advection_1d(64, stretch=0.5)
    s = mfc.Solver(spec, kernel=mfc.MFC_KERNEL_FUSED)
    q = s.upload(oracle.prim_to_cons_field(spec, w))
    s.run(q, 200, cfl=0.4)
    t, _ = s.time()
    s.check()
    qo, to, st = oracle.run(spec, oracle.prim_to_cons_field(spec, w), 200, cfl=0.4)
    assert st == oracle.OK
    assert t == pytest.approx(to, rel=1e-11)
    err = rel_l1(q.cpu().numpy(), qo, spec)
    say(f"[stretched 200 steps] sine: rel L1 {err}")
    run_parity(err, spec, oracle.prim_to_cons_field(spec, w), 200, cfl=0.4)


@pytest.mark.parametrize("kernel", sorted(KERNELS))
def test_bubble_20_steps(kernel):
    spec, w = W.bubble_collapse_3d(n=24, stretch=0.6)
    s = mfc.Solver(spec, kernel=KERNELS[kernel])
    q = s.upload(oracle.prim_to_cons_field(spec, w))
    s.run(q, 20, cfl=0.3)
    s.check()
    qi = oracle.prim_to_cons_field(spec, w)
    qo, _, st = oracle.run(spec, qi, 20, cfl=0.3)
    assert st == oracle.OK
    err = rel_l1(q.cpu().numpy(), qo, spec)
    say(f"[stretched 20 steps] bubble 24^3: rel L1 {err}")
    run_parity(err, spec, qi, 20, cfl=0.3)


@pytest.mark.parametrize("kernel", sorted(KERNELS))
def test_max_wavespeed_is_the_inverse_cfl_time_scale(kernel):
    spec, w = W.bubble_collapse_3d(n=12, stretch=0.6)
    s = mfc.Solver(spec, kernel=KERNELS[kernel])
    q = s.upload(oracle.prim_to_cons_field(spec, w))
    sm = s.max_wavespeed(q)
    _, to, st = oracle.run(spec, oracle.prim_to_cons_field(spec, w), 1, cfl=1.0)
    assert st == oracle.OK
    assert sm == pytest.approx(1.0 / to, rel=1e-13)


@pytest.mark.parametrize("kernel", sorted(KERNELS))
def test_fp32_one_step(kernel):
    spec, w = W.bubble_collapse_3d(n=(37, 21, 19), stretch=0.6)
    s = mfc.Solver(spec, precision=mfc.MFC_FP32_MIXED, kernel=KERNELS[kernel])
    q = s.upload(oracle.prim_to_cons_field(spec, w))
    s.step(q, cfl=0.3)
    s.check()
    qi = oracle.prim_to_cons_field(spec, w)
    qo, _, st = oracle.run(spec, qi, 1, cfl=0.3)
    assert st == oracle.OK
    got = q.double().cpu().numpy()
    I = spec.interior[1:]
    rho_err = np.abs((got[0] + got[1])[I] - (qo[0] + qo[1])[I]).sum() / np.abs((qo[0] + qo[1])[I]).sum()
    linf = rel_linf(got, qo, spec, floor_mom=acoustic_floor(spec, qi))
    say(f"[stretched fp32 1 step] rho L1 {rho_err:.2e}, rel Linf {linf.max():.2e}")
    assert rho_err <= 1e-6 and linf.max() <= 2e-4


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_split_stretched_reads_no_ghost_cell(prec):
    """Stretched cells on the split path with every ghost cell set to NaN:
    the right-hand side and the step (with its CFL step size from the
    non-uniform widths) are bitwise those of a filled state."""
    import torch
    spec, w = W.bubble_collapse_3d(n=(17, 15, 17), stretch=0.6)
    spec = dataclasses.replace(spec, bc=(1, 1, 0, 0, 0, 0))
    P = mfc.MFC_FP64 if prec == "fp64" else mfc.MFC_FP32_MIXED
    s = mfc.Solver(spec, kernel=mfc.MFC_KERNEL_SPLIT, precision=P)
    q = s.upload(oracle.prim_to_cons_field(spec, w))
    s.fill_ghosts(q)
    ghost = torch.ones(q.shape, dtype=torch.bool, device=q.device)
    ghost[spec.interior] = False
    qn = q.clone()
    qn[ghost] = float("nan")
    I = (slice(None),) + spec.interior[1:]
    assert torch.equal(s.rhs(q)[I], s.rhs(qn)[I])
    s.step(q, cfl=0.3)
    s.step(qn, cfl=0.3)
    s.check()
    assert torch.equal(q[I], qn[I])
