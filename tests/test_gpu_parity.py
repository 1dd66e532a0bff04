"""GPU parity: the HIP library (through its C ABI) against the FP64 CPU oracle
on the same seeded inputs.  Bars: relative L-infinity 1e-12 per variable
after one right-hand side or one SSP-RK3 step, relative L1 1e-10 per
variable after 200 steps; bitwise for the ghost fill (pure copies)."""
import sys

import numpy as np
import pytest

import oracle
from parity_util import acoustic_floor, rel_l1, rel_linf, rhs_err, rounding_spread, run_parity, step_bar
from paper_2305_09163_amd import mfc
from paper_2305_09163_amd import workloads as W

pytestmark = pytest.mark.gpu

KERNELS = {"fused": mfc.MFC_KERNEL_FUSED, "staged": mfc.MFC_KERNEL_STAGED, "split": mfc.MFC_KERNEL_SPLIT}
DEFAULT_KERNEL = mfc.MFC_KERNEL_FUSED
BENCH_KERNEL = mfc.MFC_KERNEL_SPLIT     # the path bench.py times


def say(*a):
    print(*a, file=sys.stderr, flush=True)


@pytest.fixture(scope="module", autouse=True)
def gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    mfc.lib()
    yield


def workload(name):
    if name == "shock_tube_400":
        return W.shock_tube_1d(400)
    if name == "shock_tube_37":
        return W.shock_tube_1d(37)
    if name == "droplet_2d_45x45":
        return W.droplet_shock_2d(45, W.SEED + 11)
    if name == "periodic_2d_24":
        return W.random_smooth_periodic(2, 24)
    if name == "bubble_3d_37x21x19":
        return W.bubble_collapse_3d(n=(37, 21, 19))
    if name == "bubble_3d_32":
        return W.bubble_collapse_3d(n=32)
    if name == "periodic_3d_13":
        return W.random_smooth_periodic(3, 13)
    if name == "cloud_3d_40":
        return W.bubble_cloud_3d(n=40)
    raise KeyError(name)


SMALL = ["shock_tube_37", "shock_tube_400", "droplet_2d_45x45", "periodic_2d_24", "bubble_3d_37x21x19",
         "periodic_3d_13", "cloud_3d_40"]


def needs_3d(kernel, spec):
    """The split path is built for 3D only (mfc_init_grid rejects it otherwise)."""
    if kernel == "split" and spec.ndim != 3:
        pytest.skip("the split path is 3D only")


def gpu_state(solver, w):
    """The oracle's conservative initial state, uploaded bit for bit: both
    sides start from identical inputs (the GPU's own primitive ->
    conservative conversion is checked separately, to 1e-14)."""
    return solver.upload(oracle.prim_to_cons_field(solver.spec, w))


def host(t):
    return t.detach().cpu().numpy()


@pytest.mark.parametrize("name", SMALL)
def test_prim_to_cons_parity(name):
    spec, w = workload(name)
    say(f"[prim_to_cons] {name} {spec.n}")
    s = mfc.Solver(spec, kernel=mfc.MFC_KERNEL_STAGED)
    q = host(gpu_state(s, w))
    qo = oracle.prim_to_cons_field(spec, w)
    for v in range(spec.nvar):
        den = np.abs(qo[v]).max()
        assert np.abs(q[v] - qo[v]).max() <= 1e-14 * max(den, 1e-300), v


@pytest.mark.parametrize("name", ["shock_tube_37", "periodic_2d_24", "bubble_3d_37x21x19", "periodic_3d_13"])
def test_fill_ghosts_bitwise(name):
    import torch
    spec, _ = workload(name)
    say(f"[fill_ghosts] {name} {spec.n} bc={spec.bc}")
    rng = np.random.default_rng(3)
    qh = rng.normal(size=spec.shape)
    s = mfc.Solver(spec, kernel=mfc.MFC_KERNEL_STAGED)
    q = torch.as_tensor(qh).cuda()
    s.fill_ghosts(q)
    np.testing.assert_array_equal(host(q), oracle.fill_ghosts(spec, qh))


@pytest.mark.parametrize("kernel", sorted(KERNELS))
@pytest.mark.parametrize("name", SMALL)
def test_rhs_parity(name, kernel):
    spec, w = workload(name)
    needs_3d(kernel, spec)
    say(f"[rhs] {name} {spec.n} kernel={kernel}")
    s = mfc.Solver(spec, kernel=KERNELS[kernel])
    q = gpu_state(s, w)
    s.fill_ghosts(q)
    r = host(s.rhs(q))
    s.check()
    qo = oracle.fill_ghosts(spec, oracle.prim_to_cons_field(spec, w))
    ro, st = oracle.rhs(spec, qo)
    assert st == oracle.OK
    err = rhs_err(r, ro, qo, spec)
    say(f"    CFL-step error per variable {err}")
    say(f"    rel Linf of the right-hand side, own scales {rel_linf(r, ro, spec)}")
    assert err.max() <= 1e-12, err


@pytest.mark.parametrize("kernel", sorted(KERNELS))
@pytest.mark.parametrize("name", SMALL)
def test_one_step_parity(name, kernel):
    spec, w = workload(name)
    needs_3d(kernel, spec)
    say(f"[rk3 1 step] {name} {spec.n} kernel={kernel}")
    s = mfc.Solver(spec, kernel=KERNELS[kernel])
    q = gpu_state(s, w)
    s.step(q, cfl=0.3)
    t, dt = s.time()
    s.check()
    qi = oracle.prim_to_cons_field(spec, w)
    qo, to, st = oracle.run(spec, qi, 1, cfl=0.3)
    assert st == oracle.OK
    assert dt == pytest.approx(to, rel=1e-13)
    err = rel_linf(host(q), qo, spec)
    bar = step_bar(rounding_spread(spec, qi, 1, cfl=0.3))
    say(f"    rel Linf per variable (own scales) {err}; bar {bar}")
    assert (err <= bar).all(), (err, bar)


@pytest.mark.parametrize("kernel", sorted(KERNELS))
def test_shock_tube_200_steps_parity(kernel):
    """The 1D water/air shock tube, 400 cells, CFL 0.4, 200 steps."""
    spec, w = W.shock_tube_1d(400)
    needs_3d(kernel, spec)
    say(f"[rk3 200 steps] shock_tube_400 kernel={kernel}")
    s = mfc.Solver(spec, kernel=KERNELS[kernel])
    q = gpu_state(s, w)
    s.run(q, 200, cfl=0.4)
    t, _ = s.time()
    s.check()
    qo, to, st = oracle.run(spec, oracle.prim_to_cons_field(spec, w), 200, cfl=0.4)
    assert st == oracle.OK
    assert t == pytest.approx(to, rel=1e-11)
    err = rel_l1(host(q), qo, spec)
    say(f"    rel L1 per variable {err}")
    run_parity(err, spec, oracle.prim_to_cons_field(spec, w), 200, cfl=0.4)


@pytest.mark.parametrize("kernel", sorted(KERNELS))
def test_bubble_3d_steps_parity(kernel):
    """3D bubble collapse at 32^3 (the 128^3 workload's recipe), 20 steps."""
    spec, w = W.bubble_collapse_3d(n=32)
    needs_3d(kernel, spec)
    say(f"[rk3 20 steps] bubble_3d_32 kernel={kernel}")
    s = mfc.Solver(spec, kernel=KERNELS[kernel])
    q = gpu_state(s, w)
    s.run(q, 20, cfl=0.3)
    s.check()
    qo, to, st = oracle.run(spec, oracle.prim_to_cons_field(spec, w), 20, cfl=0.3)
    assert st == oracle.OK
    err = rel_l1(host(q), qo, spec)
    say(f"    rel L1 per variable {err}")
    qi = oracle.prim_to_cons_field(spec, w)
    run_parity(err, spec, qi, 20, cfl=0.3)
    run_parity(rel_linf(host(q), qo, spec), spec, qi, 20, cfl=0.3, norm="linf")


def test_bubble_3d_200_steps_parity():
    """3D bubble collapse at 32^3, 200 steps at CFL 0.3 on the benchmark
    path: relative L1 within 1e-10 of the oracle, and the same simulated
    time."""
    spec, w = W.bubble_collapse_3d(n=32)
    say("[rk3 200 steps] bubble_3d_32 kernel=split")
    s = mfc.Solver(spec, kernel=BENCH_KERNEL)
    q = gpu_state(s, w)
    s.run(q, 200, cfl=0.3)
    t, _ = s.time()
    s.check()
    qo, to, st = oracle.run(spec, oracle.prim_to_cons_field(spec, w), 200, cfl=0.3)
    assert st == oracle.OK
    assert t == pytest.approx(to, rel=1e-11)
    err = rel_l1(host(q), qo, spec)
    say(f"    rel L1 per variable (own scales) {err}")
    run_parity(err, spec, oracle.prim_to_cons_field(spec, w), 200, cfl=0.3)


def test_full_size_bubble_one_step_parity():
    """The 128^3 bubble-collapse workload: one SSP-RK3 step at CFL 0.3 in the
    launch configuration the benchmark times, relative L-infinity within
    1e-12 of the oracle."""
    spec, w = W.bubble_collapse_3d(n=128)
    say("[rk3 1 step full size] bubble_3d_128 kernel=split")
    s = mfc.Solver(spec, kernel=BENCH_KERNEL)
    q = gpu_state(s, w)
    s.step(q, cfl=0.3)
    s.check()
    qi = oracle.prim_to_cons_field(spec, w)
    qo, _, st = oracle.run(spec, qi, 1, cfl=0.3)
    assert st == oracle.OK
    err = rel_linf(host(q), qo, spec)
    bar = step_bar(rounding_spread(spec, qi, 1, cfl=0.3))
    say(f"    rel Linf per variable (own scales) {err}; bar {bar}")
    assert (err <= bar).all(), (err, bar)


def test_max_wavespeed_parity():
    for name in ["shock_tube_400", "droplet_2d_45x45", "bubble_3d_37x21x19"]:
        spec, w = workload(name)
        say(f"[max_wavespeed] {name}")
        s = mfc.Solver(spec, kernel=mfc.MFC_KERNEL_STAGED)
        q = gpu_state(s, w)
        sm = s.max_wavespeed(q)
        so, st = oracle.max_wavespeed(spec, oracle.prim_to_cons_field(spec, w))
        assert sm == pytest.approx(so, rel=1e-14)


@pytest.mark.parametrize("kernel", ["split", "fused"])
def test_full_size_bubble_rhs_parity(kernel):
    """The 128^3 bubble-collapse workload: one full right-hand side (every
    interior cell) against the oracle; the split path is the launch
    configuration the benchmark times."""
    spec, w = W.bubble_collapse_3d(n=128)
    say(f"[rhs full size] bubble_3d_128 kernel={kernel}")
    s = mfc.Solver(spec, kernel=KERNELS[kernel])
    q = gpu_state(s, w)
    s.fill_ghosts(q)
    r = host(s.rhs(q))
    s.check()
    qo = oracle.fill_ghosts(spec, oracle.prim_to_cons_field(spec, w))
    ro, st = oracle.rhs(spec, qo)
    assert st == oracle.OK
    err = rhs_err(r, ro, qo, spec)
    say(f"    CFL-step error per variable {err}")
    say(f"    rel Linf of the right-hand side, own scales {rel_linf(r, ro, spec)}")
    assert err.max() <= 1e-12, err


def test_nonphysical_state_is_reported():
    spec, w = W.shock_tube_1d(40)
    w = w.copy()
    w[0, 0, 0, 20] = -5.0    # negative partial density of water, beyond the air share
    w[1, 0, 0, 20] = 0.0
    s = mfc.Solver(spec, kernel=mfc.MFC_KERNEL_STAGED)
    q = gpu_state(s, w)
    with pytest.raises(mfc.MfcError) as e:
        s.max_wavespeed(q)
    assert e.value.status == mfc.MFC_E_NONPHYSICAL
    s.fill_ghosts(q)
    s.rhs(q)
    with pytest.raises(mfc.MfcError) as e:
        s.check()
    assert e.value.status == mfc.MFC_E_NONPHYSICAL
    s.check()  # flag cleared


@pytest.mark.parametrize("kernel", sorted(KERNELS))
def test_nonphysical_flag_agrees_with_oracle(kernel):
    """An under-resolved bubble (about 2 cells per radius in z) whose WENO
    reconstructions leave the physical range in the first step: the oracle and
    the GPU both report it; a resolved one is clean on both."""
    for n, expect in (((24, 20, 18), True), ((36, 34, 33), False)):
        spec, w = W.bubble_collapse_3d(n=n)
        say(f"[flag] bubble {n} kernel={kernel}")
        _, _, st = oracle.run(spec, oracle.prim_to_cons_field(spec, w), 1, cfl=0.3)
        assert (st == oracle.E_NONPHYSICAL) == expect
        s = mfc.Solver(spec, kernel=KERNELS[kernel])
        q = gpu_state(s, w)
        s.step(q, cfl=0.3)
        if expect:
            with pytest.raises(mfc.MfcError) as e:
                s.check()
            assert e.value.status == mfc.MFC_E_NONPHYSICAL
        else:
            s.check()


@pytest.mark.parametrize("kernel", sorted(KERNELS))
def test_deterministic_reruns(kernel):
    spec, w = W.bubble_collapse_3d(n=(37, 21, 19))
    needs_3d(kernel, spec)
    outs = []
    for _ in range(2):
        s = mfc.Solver(spec, kernel=KERNELS[kernel])
        q = gpu_state(s, w)
        s.run(q, 3, cfl=0.3)
        outs.append(host(q))
    np.testing.assert_array_equal(outs[0], outs[1])


def test_rk3_equals_composed_primitives():
    """mfc_rk3_step equals ghost fill + rhs + the stage combinations done by hand
    (up to the fused multiply-adds of the stage update)."""
    import torch
    spec, w = W.bubble_collapse_3d(n=(37, 21, 19))
    s = mfc.Solver(spec, kernel=DEFAULT_KERNEL)
    q = gpu_state(s, w)
    q0 = q.clone()
    dt = 1e-7
    s.step(q, dt=dt)
    qs = q0.clone()
    coef = [(0.0, 1.0), (0.75, 0.25), (1.0 / 3.0, 2.0 / 3.0)]
    for a, b in coef:
        s.fill_ghosts(qs)
        L = s.rhs(qs)
        qs = a * q0 + b * (qs + dt * L)
    err = rel_linf(host(q), host(qs), spec)
    # the kernel's stage update uses fused multiply-adds, the composition
    # does not: 1e-14, or twice the oracle's own spread between those two
    # rounding orders over the same step (momentum of water at rest)
    bar = step_bar(rounding_spread(spec, oracle.prim_to_cons_field(spec, w), 1, cfl=0.0, dt=dt), 1e-14)
    assert (err <= bar).all(), (err, bar)


def test_kernel_timing_covers_the_enabled_steps_only():
    """Kernel timing switched on for some steps only: mfc_kernel_time reports
    the launches of exactly those steps (disabling keeps what was recorded)
    and resets; the timed durations are positive."""
    spec, w = W.bubble_collapse_3d(n=32)
    s = mfc.Solver(spec, kernel=mfc.MFC_KERNEL_SPLIT)
    q = s.state_from_prim(w)
    for i in range(5):
        on = i in (0, 3)
        if on:
            mfc.mfc_set_kernel_timing(s.h, True)
        s.step(q, cfl=0.3)
        if on:
            mfc.mfc_set_kernel_timing(s.h, False)
    ms0, n0 = mfc.mfc_kernel_time(s.h, 0)
    ms1, n1 = mfc.mfc_kernel_time(s.h, 1)
    assert n0 == 6 and n1 == 6          # three stages in each of the two timed steps
    assert ms0 > 0.0 and ms1 > 0.0
    assert mfc.mfc_kernel_time(s.h, 0) == (0.0, 0)
    s.check()


def test_rk3_step_reports_dt_used():
    """mfc_rk3_step writes the step size it took to the caller's device
    word: the CFL step (equal to mfc_time's last step) and a given dt."""
    import torch
    spec, w = W.bubble_collapse_3d(n=(24, 20, 18))
    for kernel in (mfc.MFC_KERNEL_SPLIT, mfc.MFC_KERNEL_FUSED):
        s = mfc.Solver(spec, kernel=kernel)
        q = gpu_state(s, w)
        d = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        s.step(q, cfl=0.3, dt_used=d)
        t, last = s.time()
        assert float(d.item()) == last and last > 0.0 and t == last
        s.step(q, dt=2.5e-7, dt_used=d)
        assert float(d.item()) == 2.5e-7
        s.step(q, cfl=0.3)   # no pointer: nothing written
        assert float(d.item()) == 2.5e-7


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("recon", ["weno5", "weno3"])
def test_run_carries_the_wave_speeds(prec, recon):
    """On the split path mfc_run has the last stage of each step reduce the
    wave speeds of the state it writes, for the next step's size.  Two steps
    of one run against two mfc_rk3_step calls: the first steps are the same
    launches but for that reduction, so the second step sizes must be equal
    bit for bit (the reduction converts the same stored values as the next
    first stage does); the states then agree to rounding (the carried first
    stage forms q + dt L_xy + dt L_z, the other q + dt (L_xy + L_z))."""
    spec, w = W.bubble_collapse_3d(n=(37, 21, 19))   # ragged tiles, two z chunks
    P = mfc.MFC_FP64 if prec == "fp64" else mfc.MFC_FP32_MIXED
    R = mfc.MFC_RECON_WENO5 if recon == "weno5" else mfc.MFC_RECON_WENO3
    a = mfc.Solver(spec, kernel=mfc.MFC_KERNEL_SPLIT, precision=P, recon=R)
    b = mfc.Solver(spec, kernel=mfc.MFC_KERNEL_SPLIT, precision=P, recon=R)
    qa, qb = gpu_state(a, w), gpu_state(b, w)
    a.run(qa, 2, cfl=0.3)
    b.step(qb, cfl=0.3)
    b.step(qb, cfl=0.3)
    a.check()
    b.check()
    ta, tb = a.time(), b.time()
    say(f"[run carries wave speeds {prec} {recon}] t {ta[0]:.17g} / {tb[0]:.17g}, "
        f"second dt {ta[1]:.17g} / {tb[1]:.17g}")
    assert ta == tb
    # momentum against rho_max c_max (the bubble starts at rest: a rounding
    # difference of the water's energy, one float ulp in FP32, moves the
    # pressure by about 1e-3 of the bubble's jump and with it the small
    # early momentum)
    floor = acoustic_floor(spec, oracle.prim_to_cons_field(spec, w))
    e = rel_linf(qa.double().cpu().numpy(), qb.double().cpu().numpy(), spec, floor_mom=floor)
    say(f"    rel Linf between the two runs {e.max():.2e}")
    assert e.max() <= (1e-13 if prec == "fp64" else 1e-5), e
