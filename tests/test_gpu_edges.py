"""Edge cases of the method against the oracle: the smallest grids (3 cells
per active dimension), uniform states (whose right-hand side is exactly
zero), fully supersonic flow in both directions (the one-sided HLLC
branches), the single-fluid Sod problem, grids that are one cell past a
tile, and the full 256^3 size checked on sampled cells, each computed by the
oracle from the 7-cell window around it."""
import dataclasses
import sys

import numpy as np
import pytest
import torch

import oracle
from parity_util import rel_linf, rhs_err, state_scales, acoustic_floor, rounding_spread, step_bar
from paper_2305_09163_amd import mfc
from paper_2305_09163_amd import workloads as W

pytestmark = pytest.mark.gpu
KERNELS = {"fused": mfc.MFC_KERNEL_FUSED, "staged": mfc.MFC_KERNEL_STAGED, "split": mfc.MFC_KERNEL_SPLIT}


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def extrapolated(sw):
    spec, w = sw
    return dataclasses.replace(spec, bc=(0, 0, 0, 0, 0, 0)), w


CASES = {
    "min_1d_3": lambda: W.random_smooth_periodic(1, 3),
    "min_2d_3": lambda: W.random_smooth_periodic(2, 3),
    "min_3d_3": lambda: W.random_smooth_periodic(3, 3),
    "min_3d_3_extrap": lambda: extrapolated(W.random_smooth_periodic(3, 3)),
    "supersonic_2d_+": lambda: W.supersonic_periodic(2, 20),
    "supersonic_2d_-": lambda: W.supersonic_periodic(2, 20, sign=-1.0),
    "supersonic_3d_-": lambda: W.supersonic_periodic(3, 12, sign=-1.0),
    "sod_1d_100": lambda: W.sod_1d(100),
    "tile_plus_one_3d": lambda: W.bubble_collapse_3d(n=(17, 15, 17)),
    "tile_plus_one_2d": lambda: W.droplet_shock_2d((17, 17), W.SEED + 21),
}


def kernels_for(spec):
    return [k for k in sorted(KERNELS) if k != "split" or spec.ndim == 3]


PAIRS = [(name, k) for name, make in CASES.items() for k in kernels_for(make()[0])]


@pytest.mark.parametrize("name,kernel", PAIRS)
def test_edge_rhs_and_step(name, kernel):
    spec, w = CASES[name]()
    say(f"[edge] {name} {spec.n} bc={spec.bc} kernel={kernel}")
    s = mfc.Solver(spec, kernel=KERNELS[kernel])
    q = s.upload(oracle.prim_to_cons_field(spec, w))
    s.fill_ghosts(q)
    r = s.rhs(q).cpu().numpy()
    s.check()
    qo = oracle.fill_ghosts(spec, oracle.prim_to_cons_field(spec, w))
    ro, st = oracle.rhs(spec, qo)
    assert st == oracle.OK
    err = rhs_err(r, ro, qo, spec)
    q1 = s.upload(oracle.prim_to_cons_field(spec, w))
    s.step(q1, cfl=0.3)
    s.check()
    qn, _, st = oracle.run(spec, oracle.prim_to_cons_field(spec, w), 1, cfl=0.3)
    assert st == oracle.OK
    e1 = rel_linf(q1.cpu().numpy(), qn, spec)
    say(f"    rhs err {err.max():.2e}, one-step rel Linf {e1.max():.2e}")
    bar = step_bar(rounding_spread(spec, oracle.prim_to_cons_field(spec, w), 1, cfl=0.3))
    assert err.max() <= 1e-12 and (e1 <= bar).all(), (e1, bar)


def test_supersonic_cases_are_supersonic():
    for name in ("supersonic_2d_+", "supersonic_2d_-", "supersonic_3d_-"):
        spec, w = CASES[name]()
        rho = w[0] + w[1]
        c = np.sqrt(1.4 * w[2 + spec.ndim] / rho)
        for d in range(spec.ndim):
            assert (np.abs(w[2 + d]) > c).all(), name


@pytest.mark.parametrize("kernel", sorted(KERNELS))
@pytest.mark.parametrize("ndim", [1, 2, 3])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_uniform_state_has_zero_rhs(kernel, ndim, prec):
    if kernel == "split" and ndim != 3:
        pytest.skip("the split path is 3D only")
    if kernel == "staged" and prec == "fp32":
        pytest.skip("the staged path is FP64 only")
    spec, w = W.uniform_state(ndim, 19)
    s = mfc.Solver(spec, kernel=KERNELS[kernel], precision=mfc.MFC_FP64 if prec == "fp64" else mfc.MFC_FP32_MIXED)
    q = s.upload(oracle.prim_to_cons_field(spec, w))
    s.fill_ghosts(q)
    r = s.rhs(q)
    s.check()
    I = (slice(None),) + spec.interior[1:]
    assert torch.count_nonzero(r[I]).item() == 0
    # a step leaves it unchanged up to the rounding of the stage combinations
    # (3/4 q + 1/4 q and 1/3 q + 2/3 q need not give q's bits back)
    q0 = q.clone()
    s.step(q, dt=1e-6)
    s.check()
    tol = 4e-16 if prec == "fp64" else 2e-7
    assert torch.allclose(q[I], q0[I], rtol=tol, atol=0.0)


# ------------------------------------------------------- full size, sampled

def oracle_cell_rhs(spec, qf, cells):
    """Oracle right-hand side of each interior cell (i, j, k) of `cells`,
    computed on the window of 3 cells around it (a grid of one interior cell
    whose ghost layers are the real neighbours; no ghost fill)."""
    nd = spec.ndim
    win = dataclasses.replace(spec, n=(1,) * nd, lo=(0.0,) * 3, hi=tuple(spec.dx[d] for d in range(3)))
    out = []
    for (i, j, k) in cells:
        sl = [slice(None), slice(k, k + 7) if nd == 3 else slice(0, 1), slice(j, j + 7) if nd >= 2 else slice(0, 1),
              slice(i, i + 7)]
        L, st = oracle.rhs(win, np.ascontiguousarray(qf[tuple(sl)]))
        assert st == oracle.OK
        out.append(L[(slice(None),) + win.interior[1:]].reshape(-1))
    return np.array(out)


def sample_cells(spec, n_random, rng):
    n = spec.n
    cells = set()
    for c in ((0, 0, 0), (n[0] - 1, n[1] - 1, n[2] - 1), (0, n[1] - 1, n[2] // 2), (n[0] // 2, 0, n[2] - 1)):
        cells.add(c)
    for _ in range(n_random):
        cells.add(tuple(int(rng.integers(0, n[d])) for d in range(3)))
    return sorted(cells)


@pytest.mark.parametrize("prec,kernel", [("fp64", "split"), ("fp32", "split"), ("fp64", "fused")])
def test_full_size_256_sampled(prec, kernel):
    """The 128^3 bubble recipe at 256^3 (the size of the learned-indicator
    workload): one right-hand side on the GPU, 250 cells recomputed by the
    oracle (random cells, grid corners and cells on the bubble surface)."""
    spec, w = W.bubble_collapse_3d(n=256)
    say(f"[256^3 sampled] {prec} {kernel}")
    P = mfc.MFC_FP64 if prec == "fp64" else mfc.MFC_FP32_MIXED
    s = mfc.Solver(spec, kernel=KERNELS[kernel], precision=P)
    q = s.upload(oracle.prim_to_cons_field(spec, w))
    s.fill_ghosts(q)
    r = s.rhs(q)
    s.check()
    qf = q.double().cpu().numpy()       # the GPU's own (FP32 or FP64) state, as the oracle's input
    rng = np.random.default_rng(5)
    cells = sample_cells(spec, 200, rng)
    # cells on the bubble surface, where every branch of the flux is exercised
    a1 = w[spec.nvar - 1][spec.interior[1:]]
    surf = np.argwhere((a1 > 0.05) & (a1 < 0.95))
    for idx in rng.choice(len(surf), size=50, replace=False):
        kz, jy, ix = surf[idx]
        cells.append((int(ix), int(jy), int(kz)))
    ro = oracle_cell_rhs(spec, qf, cells)
    rg = r.double().cpu().numpy()
    rg = np.array([rg[:, k + 3, j + 3, i + 3] for (i, j, k) in cells])
    smax, _ = oracle.max_wavespeed(spec, qf)
    dt = 0.3 * spec.dx[0] / smax
    # the measure of rhs_err (parity_util): the fluid starts at rest, so the
    # momentum rows are scaled by the acoustic momentum rho_max * c_max
    scale = state_scales(spec, qf, "max", floor_mom=acoustic_floor(spec, qf))
    err = dt * np.abs(rg - ro).max(axis=0) / scale
    say(f"    {len(cells)} cells, forward-Euler-step error per variable {err}")
    assert err.max() <= (1e-12 if prec == "fp64" else 2e-6), err


# ------------------------------------------- boundary conditions by index

@pytest.mark.parametrize("bc", [(0, 0, 0, 0, 0, 0), (1, 1, 1, 1, 1, 1), (1, 1, 0, 0, 1, 1)])
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_split_reads_no_ghost_cell(bc, prec):
    """The split kernels take neighbours past a face from the interior cell
    the ghost fill would copy there: with every ghost cell set to NaN the
    right-hand side and the step are bitwise those of a filled state, and the
    step leaves the ghost cells as they were."""
    spec, w = W.bubble_collapse_3d(n=(17, 15, 17))   # ragged in every tile dimension
    spec = dataclasses.replace(spec, bc=bc)
    say(f"[split bc by index] bc={bc} {prec}")
    P = mfc.MFC_FP64 if prec == "fp64" else mfc.MFC_FP32_MIXED
    s = mfc.Solver(spec, kernel=mfc.MFC_KERNEL_SPLIT, precision=P)
    q = s.upload(oracle.prim_to_cons_field(spec, w))
    s.fill_ghosts(q)
    ghost = torch.ones(q.shape, dtype=torch.bool, device=q.device)
    ghost[spec.interior] = False
    qn = q.clone()
    qn[ghost] = float("nan")
    I = (slice(None),) + spec.interior[1:]
    r1, r2 = s.rhs(q), s.rhs(qn)
    s.check()
    assert torch.equal(r1[I], r2[I])
    s.step(q, cfl=0.3)
    s.step(qn, cfl=0.3)
    s.check()
    assert torch.equal(q[I], qn[I])
    assert torch.isnan(qn[ghost]).all()
