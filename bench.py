#!/usr/bin/env python3
"""Throughput of the right-hand side of the two-fluid five-equation model
(WENO5-JS + HLLC + SSP-RK3) on one MI355X.

Workload: the 3D air-bubble collapse in water on 128^3 cells (7 state
variables, FP64, CFL 0.3, seeded spherical-harmonic surface noise), state
resident in HBM.  A step is one full SSP-RK3 step: the CFL wave-speed
reduction and three right-hand-side evaluations, each with its stage update
and boundary conditions (the split path applies them by index; the other
paths fill ghost layers first).  The metric is RHS cell-updates/s = interior cells x 3 stages
x steps / wall time.

One JSON line is printed.  `roofline` is measured on the dominant kernel (the
x+y kernel of the split path, or the single fused kernel) with HIP events
recorded by the library around its launches, on the launch stream, in every
tenth step of the timed region; `roofline_second_kernel` does the same for
the z + stage-update kernel of the split path.  `cpu_baseline` times the FP64 CPU
oracle on the host for one SSP-RK3 step of the same workload (single-threaded,
and with OpenMP on every host core under `all_cores`).

    python bench.py [--steps K] [--warmup W] [--n 128] [--kernel split|fused|staged]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "RHS cell-updates/s (WENO5+HLLC), FP64 vs FP32/learned at fixed L1 error"

# Algorithmic work per cell-update: the oracle's operations counted by
# running its source on a counting scalar type (tests/opcount; every +, -,
# *, / and sqrt with a state-dependent operand is one flop, operations on
# material and grid constants are not counted), asymptotic per interior cell
# of a periodic box.  3D: 2641 per right-hand side (conservative->primitive
# 28, per direction 870 = WENO5 99 x 7 + HLLC about 153 + flux differences and
# div(u) 24, the div(u) source 2) plus the stage combination 28 (7 values of
# 2, 5, 5 flops over the three stages).  2D: 1537 + 24.
FLOPS_PER_CELL_UPDATE = 2669
FLOPS_PER_CELL_UPDATE_2D = 1561
# Bytes per cell-update of one fused pass, averaged over the three stages:
# read the stage input (56 B), read q^n on stages 2 and 3 (56 B), write the
# result (56 B): (112 + 168 + 168) / 3.
BYTES_PER_CELL_UPDATE = (112 + 168 + 168) / 3
# The split path's two kernels.  x+y kernel: conservative->primitive 28, two
# directions of 870 and the stage combination 28 (it forms q + dt L_xy in
# the first stage and a q^n + b (q + dt L_xy) in the others) -> 1797 flops;
# reads the stage input (56 B) and, on stages 2-3, q^n (56 B), and writes
# that x+y part (7 values, 56 B): (112 + 168 + 168) / 3 B averaged over a
# step's three stages.  z kernel: the remaining 2669 - 1797 = 872 flops (one
# direction, the source, the z part of the update); reads the stage input
# and the x+y part, writes the result: 3 x 56 B.  In a run of CFL steps the
# step size is known before each first stage (the previous step's last z
# pass reduces the wave speeds it writes); only the run's first step reads
# its stage input a second time in the z pass, which the count leaves out.
SPLIT = {0: dict(name="k_xy (x+y reconstruction, HLLC, flux differences, x+y stage combination)", flops=1797,
                 bytes=(112 + 168 + 168) / 3),
         1: dict(name="k_z (z reconstruction, HLLC, source, stage update)", flops=2669 - 1797,
                 bytes=3 * 56)}
# The library's kernel events bracket the launches of every tenth step of
# the timed region.
KERNEL_TIMING_STRIDE = 10
# Measured HBM traffic per launch (bytes) of the split path's kernels on the
# 128^3 bubble: rocprofv3 FETCH_SIZE and WRITE_SIZE per dispatch, each
# scaled by its reading for a copy kernel of known size (FETCH_SIZE x 2.00,
# WRITE_SIZE x 1.00), averaged over the three stages of a step of a run
# (in which every first stage's z pass reads only what the others read; the
# run's first step, which reads its stage input twice, left out).  Valid
# only for the kernel sources they were taken on; any change to those files
# turns `traffic` back to null.
TRAFFIC_SOURCES = ("split.hip", "physics.h", "internal.h", "charbc.h")
TRAFFIC = {"sha256": "bcb207b46f1a439ca8171579f25553c3850d1683b220d2d12bbe837ebbe5d77d",
           ("split", "fp32", 128, 0): (126.15e6, 62.40e6),
           ("split", "fp32", 128, 1): (143.65e6, 61.50e6),
           ("split", "fp64", 128, 0): (242.79e6, 127.68e6),
           ("split", "fp64", 128, 1): (288.31e6, 123.55e6)}
PEAK_FP64_VALU = 78.6e12      # 256 CU x 2.4 GHz x 128 FP64 flop/clk/CU
PEAK_FP32_VALU = 157.3e12
PEAK_HBM = 8.0e12


def measured_traffic(kernel, precision, recon, model, stretch, n, slot, bc="extrap"):
    """(read, write) HBM bytes per launch from the counter runs (WENO5
    kernels only), or None."""
    import hashlib
    if recon != "weno5" or model != "allaire" or stretch or bc != "extrap":
        return None
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2305_09163_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest() != TRAFFIC["sha256"]:
        return None
    return TRAFFIC.get((kernel, precision, n, slot))


def reference_run(spec, w, steps, mfc):
    """The FP64 WENO5 path (the one the parity tests check against the
    oracle) advanced `steps` steps of one fixed dt, CFL 0.3 of the initial
    state; the forms are compared with it after the same steps."""
    ref = mfc.Solver(spec, kernel=mfc.MFC_KERNEL_SPLIT if spec.faces is None else mfc.MFC_KERNEL_FUSED,
                     precision=mfc.MFC_FP64)
    qr = ref.state_from_prim(w)
    dt = 0.3 * min(spec.dx[:spec.ndim]) / ref.max_wavespeed(qr)
    ref.run(qr, steps, dt=dt)
    ref.check()
    return ref, qr, dt


def error_vs_reference(spec, w, make_solver, steps, mfc, weights, tau, reference=None):
    """Relative L1 density error of this form against the FP64 WENO5 path
    after `steps` steps of one fixed dt from the same initial state; with a
    network, also the share of interior (cell, direction) reconstructions it
    routes to the linear stencil at the end."""
    ref, qr, dt = reference or reference_run(spec, w, steps, mfc)
    s = make_solver()
    q = s.state_from_prim(w)
    s.run(q, steps, dt=dt)
    s.check()
    I = (slice(None),) + spec.interior[1:]
    rho_r = (qr[0] + qr[1])[I[1:]].double()
    rho = (q[0] + q[1])[I[1:]].double()
    out = {"rel_l1_density": float((rho - rho_r).abs().sum() / rho_r.abs().sum()), "steps": steps, "dt": dt,
           "reference": "FP64 WENO5 split path (parity-tested against the oracle)"}
    if weights is not None:
        X, Y, _ = ref.harvest(q.double().contiguous())
        t = mfc.Trainer(1)
        t.set_params(weights)
        P = t.infer(X)
        out.update(routed_to_linear=float((P > tau).float().mean()), labelled_smooth=float(Y.float().mean()))
    return out


def timed_run(torch, mfc, solver, q, steps, warmup, cfl):
    """Advance q by `warmup` untimed and `steps` timed SSP-RK3 steps, the
    timed ones as one run (mfc_run: on the split path each step's size comes
    from the wave speeds its predecessor's last stage reduced); the library's
    kernel events cover every KERNEL_TIMING_STRIDE-th timed step (events
    between all launches would lengthen every step by about 4 %).  Returns
    the elapsed seconds and (ms, launches) of both kernel slots."""
    solver.run(q, warmup, cfl=cfl)
    torch.cuda.synchronize()
    solver.check()
    mfc.mfc_kernel_time(solver.h, 0)   # nothing recorded before the timed region
    mfc.mfc_kernel_time(solver.h, 1)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    mfc.mfc_set_kernel_timing(solver.h, True, KERNEL_TIMING_STRIDE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    solver.run(q, steps, cfl=cfl)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    mfc.mfc_set_kernel_timing(solver.h, False)
    k0 = mfc.mfc_kernel_time(solver.h, 0)
    k1 = mfc.mfc_kernel_time(solver.h, 1)
    solver.check()
    return max(wall, e0.elapsed_time(e1) / 1e3), k0, k1


def cpu_baseline(spec, w, workload="bubble"):
    """The FP64 oracle on the host for one SSP-RK3 step of the same workload:
    the plain single-threaded build, and the OpenMP build of the same source
    on every host core it is given (OMP_NUM_THREADS, else all cores).  Above
    128^3 cells the sample is the same workload generated at 128^3 (one step
    of 256^3 takes the single-threaded oracle about 40 s)."""
    import oracle
    from paper_2305_09163_amd import workloads as W

    name = "bubble cloud" if workload == "cloud" else "bubble"
    if spec.cells > 128 ** 3 and spec.faces is None:
        import dataclasses
        gen = W.bubble_cloud_3d if workload == "cloud" else W.bubble_collapse_3d
        s2, w = gen(n=128)
        spec = dataclasses.replace(s2, model=spec.model, bc=spec.bc)

    def one_step():
        q = oracle.prim_to_cons_field(spec, w)
        t0 = time.perf_counter()
        _, _, st = oracle.run(spec, q, 1, cfl=0.3)
        el = time.perf_counter() - t0
        assert st == oracle.OK
        return el

    el = one_step()
    with oracle.threaded() as threads:
        el_t = one_step()
    sample = f"1 SSP-RK3 step (3 RHS evaluations) of the {spec.n[0]}^3 {name} workload"
    return {"value": spec.cells * 3 / el, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{sample}, single-threaded C oracle (gcc -O2), {el:.1f} s",
            "host_cpus": os.cpu_count(),
            "all_cores": {"value": spec.cells * 3 / el_t, "unit": "cell-updates/s", "cores": threads,
                          "kind": "oracle",
                          "sample": f"{sample}, the same oracle built with OpenMP over the pencils of each "
                                    f"sweep, {threads} threads, {el_t:.2f} s"}}


def bench_ensemble(args, torch, mfc, W):
    """64 independent 2D droplet-shock runs (N^2 cells, N = 64 .. 512, seeded),
    FP32 storage form, advanced together by the batch path (autotuned launch
    configuration, graph replay) and, for comparison, one run after another
    through the single-grid fused path.  Both are timed over the same steps;
    the batch is bitwise equal to the sequential runs."""
    sizes = W.ensemble_sizes()
    runs = [W.droplet_shock_2d(n, W.SEED + 1000 + i) for i, n in enumerate(sizes)]
    specs = [s for s, _ in runs]
    cfl = 0.3
    b = mfc.Batch(specs, precision=mfc.MFC_FP32_MIXED)
    qs = b.states_from_prim([w for _, w in runs])
    q_seq = [q.clone() for q in qs]
    best, table = b.autotune(qs, reps=5)
    b.run(qs, args.warmup, cfl, use_graph=True)
    torch.cuda.synchronize()
    b.check()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    b.run(qs, args.steps, cfl, use_graph=True)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    elapsed = max(wall, e0.elapsed_time(e1) / 1e3)
    b.check()
    updates = b.cells * 3 * args.steps
    # the stage kernel alone, timed with events on an eager pass of the same length
    mfc.mfc_batch_set_timing(b.b, True)
    b.run(qs, args.steps, cfl, use_graph=False)
    ms_k, n_k = mfc.mfc_batch_kernel_time(b.b)
    mfc.mfc_batch_set_timing(b.b, False)
    b.check()
    avg = ms_k / 1e3 / max(n_k, 1)
    # sequential per-run launches through the single-grid fused path
    solvers = [mfc.Solver(sp, precision=mfc.MFC_FP32_MIXED, kernel=mfc.MFC_KERNEL_FUSED) for sp in specs]
    for s, q in zip(solvers, q_seq):
        s.run(q, args.warmup, cfl=cfl)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, q in zip(solvers, q_seq):
        s.run(q, args.steps, cfl=cfl)
    torch.cuda.synchronize()
    seq = time.perf_counter() - t0
    # 2D algorithmic work per cell-update (counted on the oracle, above).
    # Bytes (FP32, 6 values of 4 B): read the stage input, read q^n on
    # stages 2-3, write the result.
    flops = FLOPS_PER_CELL_UPDATE_2D
    nbytes = (2 * 24 + 3 * 24 + 3 * 24) / 3
    bound = "alu" if flops / nbytes > PEAK_FP32_VALU / PEAK_HBM else "hbm"
    ach = flops * b.cells / avg
    roof = {"bound": bound, "achieved": ach / 1e12, "peak": PEAK_FP32_VALU / 1e12, "unit": "TFLOP/s",
            "frac": ach / PEAK_FP32_VALU, "traffic": None,
            "kernel": "k_batch_stage (2D right-hand side + stage update, all runs)", "launches": n_k,
            "avg_launch_us": avg * 1e6, "flops_per_cell_update": flops, "bytes_per_cell_update": nbytes,
            "hbm_algorithmic_GBps": nbytes * b.cells / avg / 1e9,
            "timed_on": "eager pass of the same length right after the graph-timed region"}
    out = {"metric": METRIC, "value": updates / elapsed, "unit": "cell-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
           "data": "synthetic",
           "config": {"workload": "droplet_shock_2d_ensemble_64", "runs": len(sizes), "cells": b.cells,
                      "sizes": sizes, "cfl": cfl, "precision": "fp32", "tune": dict(zip(("shape", "groups", "xcd"), best)),
                      "tile": mfc.BATCH_SHAPES[best[0]], "parallelism": "single GPU"},
           "sequential_single_grid": {"value": updates / seq, "ms_per_step": seq / args.steps * 1e3,
                                      "speedup_of_batch": seq / elapsed},
           "autotune_ms": table, "roofline": roof}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=128)
    ap.add_argument("--kernel", choices=["fused", "staged", "split"], default="split")
    ap.add_argument("--precision", choices=["fp64", "fp32"], default="fp64")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", choices=["bubble", "cloud", "ensemble"], default="bubble",
                    help="bubble: the 3D bubble collapse (default); cloud: 50 bubbles struck by a pressure "
                         "step (3D, use --n 256 --precision fp32 --steps 50); ensemble: 64 uneven 2D "
                         "droplet-shock runs")
    ap.add_argument("--no-forms", action="store_true",
                    help="time only the requested form (the default FP64 line also times the FP32 and "
                         "learned forms)")
    ap.add_argument("--recon", choices=["weno5", "learned", "weno3", "first"], default="weno5",
                    help="learned: reconstruction routed by the trained indicator (weights from --weights); "
                         "weno3 / first: the third- and first-order reconstructions")
    ap.add_argument("--model", choices=["allaire", "kapila"], default="allaire",
                    help="volume-fraction equation: Allaire (default) or Kapila (with the K div(u) source)")
    ap.add_argument("--stretch", type=float, default=0.0,
                    help="tanh stretching depth of the grid around the bubble (0: uniform; split or fused kernel)")
    ap.add_argument("--bc", choices=["extrap", "characteristic"], default="extrap",
                    help="boundary of all six faces: zero-gradient extrapolation (default) or the "
                         "characteristic non-reflecting form")
    ap.add_argument("--tau", type=float, default=None,
                    help="routing threshold on P(smooth) (default: the one stored beside the weights, else 0.5)")
    ap.add_argument("--weights", default=os.path.join(ROOT, "paper_2305_09163_amd", "indicator_weights.npy"))
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="after the run, scale-copy MIB MiB of float64 three times (a kernel of known HBM "
                         "traffic that calibrates the FETCH_SIZE / WRITE_SIZE counters)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py: runs on one GPU (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the path runs on one GPU; sharding across GPUs is not built", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2305_09163_amd import mfc
    from paper_2305_09163_amd import workloads as W

    torch.cuda.set_device(0)
    if args.workload == "ensemble":
        return bench_ensemble(args, torch, mfc, W)
    if args.stretch > 0.0 and args.kernel == "staged":
        sys.exit("bench.py: stretched grids run on the split or the fused kernel")
    if args.workload == "cloud":
        spec, w = W.bubble_cloud_3d(n=args.n)
    else:
        spec, w = W.bubble_collapse_3d(n=args.n, stretch=args.stretch)
    if args.model == "kapila":
        import dataclasses
        spec = dataclasses.replace(spec, model=1)
    if args.bc == "characteristic":
        import dataclasses
        spec = dataclasses.replace(spec, bc=(mfc.MFC_BC_CHARACTERISTIC,) * 6)
    kernels = {"fused": mfc.MFC_KERNEL_FUSED, "staged": mfc.MFC_KERNEL_STAGED, "split": mfc.MFC_KERNEL_SPLIT}
    precisions = {"fp64": mfc.MFC_FP64, "fp32": mfc.MFC_FP32_MIXED}
    recons = {"weno5": mfc.MFC_RECON_WENO5, "learned": mfc.MFC_RECON_LEARNED, "weno3": mfc.MFC_RECON_WENO3,
              "first": mfc.MFC_RECON_FIRST_ORDER}
    # the default line (FP64 WENO5 on the split kernels) also times the FP32
    # and learned forms on the same workload: the metric compares them
    default_form = (args.kernel == "split" and args.precision == "fp64" and args.recon == "weno5"
                    and args.model == "allaire" and args.stretch == 0.0 and args.bc == "extrap")
    compare = default_form and not args.no_forms
    learned = args.recon == "learned" or compare
    weights = None
    if learned:
        import numpy as np
        if not os.path.exists(args.weights):
            sys.exit(f"bench.py: {args.weights} not found; train it with "
                     "`python -m paper_2305_09163_amd.train_indicator`")
        weights = np.load(args.weights, allow_pickle=False)
        if args.tau is None:
            meta = os.path.splitext(args.weights)[0] + ".json"
            args.tau = json.load(open(meta))["tau"] if os.path.exists(meta) else 0.5

    def solver_factory(precision, recon):
        def make():
            s = mfc.Solver(spec, kernel=kernels[args.kernel], precision=precisions[precision],
                           recon=recons[recon])
            if recon == "learned":
                s.set_indicator(weights, args.tau)
            return s
        return make

    make_solver = solver_factory(args.precision, args.recon)
    solver = make_solver()
    q = solver.state_from_prim(w)
    cfl = 0.3
    elapsed, (ms_kernel, launches), (ms_kernel1, launches1) = timed_run(torch, mfc, solver, q, args.steps,
                                                                        args.warmup, cfl)
    updates = spec.cells * 3 * args.steps
    value = updates / elapsed

    def roofline(ms, n, name, flops, nbytes, precision, slot=0):
        # the FP32 form's arithmetic is FP32 except the pressure recovery and s*
        peak_alu = PEAK_FP64_VALU if precision == "fp64" else PEAK_FP32_VALU
        nbytes = nbytes * (1.0 if precision == "fp64" else 0.5)  # byte counts above are for 8-byte values
        avg = ms / 1e3 / max(n, 1)
        achieved = flops * spec.cells / avg
        hbm = nbytes * spec.cells / avg
        bound = "alu" if flops / nbytes > peak_alu / PEAK_HBM else "hbm"
        r = {"bound": bound, "achieved": achieved / 1e12, "peak": peak_alu / 1e12, "unit": "TFLOP/s",
             "frac": achieved / peak_alu, "traffic": None}
        if bound == "hbm":
            r.update(achieved=hbm / 1e9, peak=PEAK_HBM / 1e9, unit="GB/s", frac=hbm / PEAK_HBM)
        tr = measured_traffic(args.kernel, precision, args.recon, args.model, args.stretch, args.n, slot,
                              args.bc) if args.workload == "bubble" else None
        if tr:
            # measured HBM bytes per launch over the same average launch duration
            r.update(traffic=sum(tr) / avg / 1e9, traffic_unit="GB/s",
                     traffic_bytes_per_launch={"read": tr[0], "write": tr[1]},
                     traffic_vs_algorithmic=sum(tr) / (nbytes * spec.cells))
        r.update({"kernel": name, "launches": n, "timed_steps": f"every {KERNEL_TIMING_STRIDE}th step of the timed region",
                  "avg_launch_us": avg * 1e6, "flops_per_cell_update": flops,
                  "bytes_per_cell_update": nbytes, "alu_TFLOPs": achieved / 1e12, "alu_frac": achieved / peak_alu,
                  "hbm_algorithmic_GBps": hbm / 1e9, "hbm_frac": hbm / PEAK_HBM})
        return r

    if args.kernel == "split":
        roof = roofline(ms_kernel, launches, SPLIT[0]["name"], SPLIT[0]["flops"], SPLIT[0]["bytes"], args.precision)
        roof_z = roofline(ms_kernel1, launches1, SPLIT[1]["name"], SPLIT[1]["flops"], SPLIT[1]["bytes"],
                          args.precision, slot=1)
    else:
        name = "k_fused<3> (fused RHS + stage update)" if args.kernel == "fused" else "staged RHS sequence"
        roof = roofline(ms_kernel, launches, name, FLOPS_PER_CELL_UPDATE, BYTES_PER_CELL_UPDATE, args.precision)
        roof_z = None
    t, _ = solver.time()
    out = {"metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f64" if args.precision == "fp64" else "f32+f64",
           "data": "synthetic",
           "config": {"workload": f"{'bubble_cloud' if args.workload == 'cloud' else 'bubble_collapse'}_3d_{args.n}",
                      "cells": spec.cells, "nvar": spec.nvar,
                      "cfl": cfl, "precision": args.precision, "kernel": args.kernel, "recon": args.recon,
                      "model": args.model, "stretch": args.stretch, "bc": args.bc,
                      "parallelism": "single GPU"},
           "roofline": roof, "simulated_time_s": t, "cell_steps_per_s": value / 3}
    if args.recon == "learned":
        out["config"]["tau"] = args.tau
    if roof_z:
        out["roofline_second_kernel"] = roof_z
    reference = None
    if args.precision == "fp32" or args.recon != "weno5" or compare:
        reference = reference_run(spec, w, args.steps, mfc)
    if args.precision == "fp32" or args.recon != "weno5":
        out["error_vs_fp64_weno5"] = error_vs_reference(spec, w, make_solver, args.steps, mfc,
                                                        weights if args.recon == "learned" else None, args.tau,
                                                        reference)
    if compare:
        # the metric's comparison: each form timed on the same workload and
        # steps, its rate against this line's FP64 rate, and its relative L1
        # density error against the FP64 path after the same steps
        forms = {}
        for precision, recon in (("fp32", "weno5"), ("fp64", "learned"), ("fp32", "learned")):
            mk = solver_factory(precision, recon)
            s2 = mk()
            q2 = s2.state_from_prim(w)
            el2, (msa, na), (msb, nb) = timed_run(torch, mfc, s2, q2, args.steps, args.warmup, cfl)
            v2 = updates / el2
            f = {"value": v2, "unit": "cell-updates/s", "ms_per_step": el2 / args.steps * 1e3,
                 "ratio_to_fp64": v2 / value, "precision": precision, "recon": recon,
                 "kernel_avg_launch_us": {"k_xy": msa / max(na, 1) * 1e3, "k_z": msb / max(nb, 1) * 1e3}}
            if recon == "learned":
                f["tau"] = args.tau
            f.update(error_vs_reference(spec, w, mk, args.steps, mfc, weights if recon == "learned" else None,
                                        args.tau, reference))
            f["meets_target"] = bool(f["ratio_to_fp64"] >= 1.8 and f["rel_l1_density"] <= 1e-4)
            forms[f"{precision}_{recon}"] = f
            del s2, q2
        out["forms"] = forms
        out["forms_target"] = "ratio_to_fp64 >= 1.8 at rel_l1_density <= 1e-4 against the FP64 path"
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(spec, w, args.workload)
    print(json.dumps(out), flush=True)
    if args.copy_probe:
        copy_probe(torch, args.copy_probe)


def copy_probe(torch, mib):
    a = torch.ones(mib * 2 ** 20 // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 2.0, out=b)
    torch.cuda.synchronize()


if __name__ == "__main__":
    main()
