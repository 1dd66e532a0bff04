"""Batched ensembles of uneven 2D runs.  The batch executes, for every run,
the arithmetic of the single-grid fused path (which the parity tests check
against the oracle), so a batched run must give the same bits as that run
advanced alone; one run is also checked against the oracle directly."""
import sys

import numpy as np
import pytest
import torch

import oracle
from parity_util import acoustic_floor, rel_l1, rel_linf, rounding_spread, run_parity, step_bar
from paper_2305_09163_amd import mfc
from paper_2305_09163_amd import workloads as W

pytestmark = pytest.mark.gpu

PREC = {"fp32": mfc.MFC_FP32_MIXED, "fp64": mfc.MFC_FP64}
SIZES = [(19, 23), (33, 27), (40, 40), (47, 29), (64, 35)]


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def ensemble(sizes, seed0=100):
    return [W.droplet_shock_2d(n, W.SEED + seed0 + i) for i, n in enumerate(sizes)]


def interior(q):
    """Interior cells of a 2D state [v, 1, py, px] (ghost cells after a step
    hold whatever the last fill left: not part of the result)."""
    return q[:, :, 3:-3, 3:-3]


def single_runs(runs, prec, nsteps, cfl=0.3):
    out = []
    for spec, w in runs:
        s = mfc.Solver(spec, precision=PREC[prec], kernel=mfc.MFC_KERNEL_FUSED)
        q = s.state_from_prim(w)
        s.run(q, nsteps, cfl=cfl)
        s.check()
        out.append((q, s.time()[0]))
        s.close()
    return out


@pytest.mark.parametrize("prec", sorted(PREC))
def test_batch_matches_single_grid_runs_bitwise(prec):
    say(f"[batch vs single] prec={prec} sizes={SIZES}")
    runs = ensemble(SIZES)
    b = mfc.Batch([s for s, _ in runs], precision=PREC[prec])
    qs = b.states_from_prim([w for _, w in runs])
    b.run(qs, 10, 0.3, use_graph=False)
    b.check()
    times = b.time()
    for r, ((q1, t1), q, t) in enumerate(zip(single_runs(runs, prec, 10), qs, times)):
        assert torch.equal(interior(q), interior(q1)), f"run {r} differs from the single-grid path"
        assert t == t1 and t > 0.0, (r, t, t1)


def test_batch_fp64_against_oracle():
    spec, w = W.droplet_shock_2d((19, 23), W.SEED + 100)
    say("[batch vs oracle] droplet 19x23 fp64, 1 and 3 steps")
    b = mfc.Batch([spec], precision=mfc.MFC_FP64)
    qi = oracle.prim_to_cons_field(spec, w)
    q = b.upload([qi])[0]
    done = 0
    for n in (1, 3):
        b.run([q], n - done, 0.3, use_graph=False)
        done = n
        b.check()
        qo, t, st = oracle.run(spec, qi, n, cfl=0.3)
        assert st == oracle.OK
        err = rel_linf(q.cpu().numpy(), qo, spec)
        bar = step_bar(rounding_spread(spec, qi, n, cfl=0.3), 1e-12 * n)
        say(f"    {n} steps rel Linf {err.max():.3e}")
        assert (err <= bar).all(), (err, bar)
        assert abs(b.time()[0] - t) <= 1e-14 * t


def test_every_launch_configuration_gives_the_same_bits():
    runs = ensemble(SIZES[:4], seed0=200)
    b = mfc.Batch([s for s, _ in runs])
    q0 = b.states_from_prim([w for _, w in runs])
    ref = None
    for shape in range(3):
        for groups in range(3):
            for xcd in range(2):
                say(f"[batch tune] shape={mfc.BATCH_SHAPES[shape]} groups/CU={mfc.BATCH_GROUPS_PER_CU[groups]} xcd={xcd}")
                qs = [q.clone() for q in q0]
                b.set_tune(shape, groups, xcd)
                b.run(qs, 3, 0.3, use_graph=False)
                b.check()
                if ref is None:
                    ref = qs
                else:
                    for r in range(len(qs)):
                        assert torch.equal(qs[r], ref[r]), (shape, groups, xcd, r)


def test_graph_replays_match_eager_steps():
    """Graph replays (4 steps each), with other eager device work and host
    synchronisation between them, against eager steps of a twin batch."""
    runs = ensemble(SIZES, seed0=300)
    specs = [s for s, _ in runs]
    bg, be = mfc.Batch(specs), mfc.Batch(specs)
    qg = bg.states_from_prim([w for _, w in runs])
    qe = [q.clone() for q in qg]
    for rep in range(3):
        say(f"[batch graph] replay {rep}")
        bg.run(qg, 4, 0.3, use_graph=True)
        junk = torch.randn(1 << 16, device="cuda").sum()  # unrelated eager work
        torch.cuda.synchronize()
        be.run(qe, 4, 0.3, use_graph=False)
        bg.check()
        be.check()
        for r in range(len(qg)):
            assert torch.equal(qg[r], qe[r]), (rep, r)
        assert bg.time() == be.time()
        del junk
    # a run that is not a multiple of the captured chunk
    bg.run(qg, 6, 0.3, use_graph=True)
    be.run(qe, 6, 0.3, use_graph=False)
    for r in range(len(qg)):
        assert torch.equal(qg[r], qe[r]), r


def test_autotune_leaves_states_and_times_alone():
    runs = ensemble(SIZES, seed0=400)
    b = mfc.Batch([s for s, _ in runs])
    qs = b.states_from_prim([w for _, w in runs])
    b.run(qs, 2, 0.3)
    before = [q.clone() for q in qs]
    t_before = b.time()
    best, table = b.autotune(qs, reps=3)
    say(f"[batch autotune] best {best} table {np.round(table, 4)}")
    assert 0 <= best[0] < 3 and 0 <= best[1] < 3 and best[2] in (0, 1)
    assert b.tune() == best
    assert all(t > 0 for t in table)
    assert min(table) == table[(best[0] * 3 + best[1]) * 2 + best[2]]
    assert b.time() == t_before
    for q, q1 in zip(qs, before):
        # ghosts are refilled from the interior, which is unchanged
        I = (slice(None), slice(None), slice(3, -3), slice(3, -3))
        assert torch.equal(q[I], q1[I])


def test_nonphysical_run_is_reported():
    runs = ensemble(SIZES[:3], seed0=500)
    b = mfc.Batch([s for s, _ in runs])
    qs = b.states_from_prim([w for _, w in runs])
    qs[1][0, 0, 10, 10] = -1.0  # negative partial density in run 1
    qs[1][1, 0, 10, 10] = -1.0
    b.step(qs, 0.3)
    with pytest.raises(mfc.MfcError) as e:
        b.check()
    assert e.value.status == mfc.MFC_E_NONPHYSICAL
    b.check()  # the flag is cleared


def test_full_ensemble_sampled_runs_match_single_grid():
    """The 64-run ensemble (N from 64 to 512) in FP32 with graph replay:
    the smallest, the largest and a middle run match the single-grid path."""
    sizes = W.ensemble_sizes()
    runs = [W.droplet_shock_2d(n, W.SEED + 1000 + i) for i, n in enumerate(sizes)]
    b = mfc.Batch([s for s, _ in runs])
    cells, nrun = b.cells, b.nrun
    say(f"[batch full] {nrun} runs, {cells} cells")
    assert nrun == 64 and cells == sum(n * n for n in sizes)
    qs = b.states_from_prim([w for _, w in runs])
    b.autotune(qs, reps=2)
    b.run(qs, 5, 0.3, use_graph=True)
    b.check()
    order = np.argsort(sizes)
    for r in (int(order[0]), int(order[-1]), int(order[32])):
        (q1, t1), = single_runs([runs[r]], "fp32", 5)
        assert torch.equal(interior(qs[r]), interior(q1)), r
        assert b.time()[r] == t1


def test_run_equals_single_steps_and_reads_no_ghost_cell():
    """mfc_batch_run takes each step's size from the wave speeds its
    predecessor's last stage reduced; single mfc_batch_step calls reduce them
    at the start of every step: the same sizes and states, bit for bit.  The
    stage kernel reads neighbours past a face through the boundary rule, so
    NaN in every ghost cell changes nothing and stays where it is."""
    runs = ensemble(SIZES, seed0=600)
    specs = [s for s, _ in runs]
    br, bs = mfc.Batch(specs), mfc.Batch(specs)
    qr = br.states_from_prim([w for _, w in runs])
    qs = [q.clone() for q in qr]
    ghost = []
    for q in qr:
        g = torch.ones(q.shape, dtype=torch.bool, device=q.device)
        g[:, :, 3:-3, 3:-3] = False
        q[g] = float("nan")
        ghost.append(g)
    br.run(qr, 5, 0.3, use_graph=False)
    for _ in range(5):
        bs.step(qs, 0.3)
    br.check()
    bs.check()
    say(f"[batch run vs steps] times {br.time()[:2]} / {bs.time()[:2]}")
    assert br.time() == bs.time()
    for r in range(len(qr)):
        assert torch.equal(interior(qr[r]), interior(qs[r])), r
        assert torch.isnan(qr[r][ghost[r]]).all(), r


def _with_bc(sw, bc):
    import dataclasses
    spec, w = sw
    return dataclasses.replace(spec, bc=bc), w


CHAR_RUNS = [
    _with_bc(W.droplet_shock_2d((19, 23), W.SEED + 700), (2, 2, 2, 2, 0, 0)),
    _with_bc(W.droplet_shock_2d((33, 27), W.SEED + 701), (2, 0, 0, 2, 0, 0)),
    _with_bc(W.droplet_shock_2d((24, 40), W.SEED + 702), (1, 1, 2, 2, 0, 0)),
    _with_bc(W.droplet_shock_2d((40, 17), W.SEED + 703), (0, 0, 0, 0, 0, 0)),
]


def test_batch_characteristic_faces_match_oracle():
    """Characteristic faces (Sec. 3.3) in batched runs, beside runs without
    them: the stage kernel takes the boundary cells' characteristic rates in
    place of their normal terms, as the oracle does; each run after 1 and 20
    steps against the oracle's run of the same run (FP64)."""
    specs = [s for s, _ in CHAR_RUNS]
    b = mfc.Batch(specs, precision=mfc.MFC_FP64)
    qi = [oracle.prim_to_cons_field(s, w) for s, w in CHAR_RUNS]
    qs = b.upload(qi)
    done = 0
    for n in (1, 20):
        b.run(qs, n - done, 0.3, use_graph=n > 1)
        done = n
        b.check()
        for r, (spec, _) in enumerate(CHAR_RUNS):
            qo, t, st = oracle.run(spec, qi[r], n, cfl=0.3)
            assert st == oracle.OK
            got = qs[r].cpu().numpy()
            if n == 1:
                err = rel_linf(got, qo, spec)
                bar = step_bar(rounding_spread(spec, qi[r], 1, cfl=0.3))
                say(f"[batch characteristic] run {r} bc={spec.bc[:4]}: one step rel Linf {err.max():.2e}")
                assert (err <= bar).all(), (r, err, bar)
            else:
                e = rel_l1(got, qo, spec)
                say(f"[batch characteristic] run {r}: {n} steps rel L1 {e.max():.2e}")
                run_parity(e, spec, qi[r], n, cfl=0.3)
            assert abs(b.time()[r] - t) <= 1e-13 * t


def test_batch_characteristic_faces_fp32():
    specs = [s for s, _ in CHAR_RUNS]
    b = mfc.Batch(specs, precision=mfc.MFC_FP32_MIXED)
    qi = [oracle.prim_to_cons_field(s, w) for s, w in CHAR_RUNS]
    qs = b.upload(qi)
    b.run(qs, 20, 0.3)
    b.check()
    for r, (spec, _) in enumerate(CHAR_RUNS):
        qo, _, st = oracle.run(spec, qi[r], 20, cfl=0.3)
        assert st == oracle.OK
        e = rel_l1(qs[r].double().cpu().numpy(), qo, spec, floor_mom=acoustic_floor(spec, qi[r]))
        say(f"[batch characteristic fp32] run {r}: rel L1 {e.max():.2e}")
        assert e.max() <= 1e-4, (r, e)
