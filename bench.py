#!/usr/bin/env python
"""Benchmark of the RT-EOM-CCSD hot path on one MI355X.

A "step" is one time step of Eq. trapzrule: ``passes`` residual evaluations
R(T) (Eqs. dt1eom/dt2eom), the fused trapezoid updates, the energy reduction
and the C(t) append, on the synthetic workload named below with all inputs
resident in HBM.  Prints one JSON line (see the design doc for every field).

    python bench.py [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from synthetic import (ESCA, ESCA_PAPER, FORMALDEHYDE, TINY, ZN_PORPHYRIN, Shape, batched_shapes,  # noqa: E402
                       draw_system)

# Ladder kernel per precision (the contraction's MFMA instruction family)
KERNEL_NAME = {"fp64": "gemm_mfma<double>", "fp32": "gemm_mfma<float> (operands converted to float planes)",
               "bf16x3": "gemm_bf16x3_split<bf16> (operands split into bf16 hi/lo planes)",
               "fp16x3": "gemm_bf16x3_split<f16> (operands scaled per row, split into fp16 hi/lo planes)"}

# HBM bytes per ladder launch from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE,
# scaled by the same counters read on a plain device copy of known size; the
# summaries (with the commands) are under profiles/.  Only workloads whose
# ladder kernel has been counted since its last change are listed.
TRAFFIC = {
    # profiles/gemm_mfma_ladder_esca_fp64.md: FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, mean of the
    # alpha-beta and same-spin ladder launches
    ("esca", "fp64"): (2.332e12, "profiles/gemm_mfma_ladder_esca71_fp64.md: FETCH_SIZE x2.000 + WRITE_SIZE x1.000, "
                                 "mean of the 82 counted ladder launches (integral slabs of 16)"),
    ("esca36", "fp64"): (7.94e11, "profiles/gemm_mfma_ladder_esca_fp64.md (o=36, v=324; kernel unchanged since)"),
}

DTYPE = {"fp64": "f64", "fp32": "f32 contractions, f64 update",
         "bf16x3": "bf16x3 contractions (f32 accumulate), f64 update",
         "fp16x3": "fp16x3 contractions (row-scaled, f32 accumulate), f64 update"}

# Matrix-core flops executed per useful flop: the split precisions run three 16-bit
# products (hi*hi, hi*lo, lo*hi) per product; their roofline counts executed flops
EXEC_PER_USEFUL = {"fp64": 1.0, "fp32": 1.0, "bf16x3": 3.0, "fp16x3": 3.0}

# Conservative residual rates (TFLOP/s) used only to fit the large workloads' steps into the budget
RATE_GUESS = {"fp64": 40.0, "fp32": 70.0, "bf16x3": 100.0, "fp16x3": 100.0}

# MI355X published peaks (dense)
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0, "fp16x3": 2500.0}
PEAK_HBM_GBS = 8000.0

# Cholesky vectors of the paper-shaped workloads are scaled by (16/v)^(1/2) (same seeds):
# drawn literally, their correlation is far beyond a molecule's (dt lambda_max / 2 of the
# (ae|bf) supermatrix 1.5 at the formaldehyde shape, 5.2 at o=36, v=324), the fixed point
# of Eq. trapzrule is no contraction there and the amplitudes overflow within tens of steps.
def chol_scale(shape):
    return (16.0 / shape.v) ** 0.5


WORKLOADS = {
    "formaldehyde": dict(shape=FORMALDEHYDE, cfg=1, dt=0.025, passes=2, steps=4,
                         desc="formaldehyde-shaped core hole: o=8, v=110 per spin, Q=600, L scaled by (16/v)^(1/2), "
                              "beta hole, dt=0.025 au"),
    "batched": dict(batch=16, cfg=2, dt=0.025, passes=2, fp_map=1, steps=10, cpu_sample="formaldehyde",
                    desc="16 independent core holes of uneven shape (o in [5,20], v in [40,200] per spin, "
                         "Q = 4 v, L scaled by (16/v)^(1/2), beta holes), diagonal fixed-point map, every "
                         "system's captured time step replayed on its own stream, dt=0.025 au"),
    "tiny": dict(shape=TINY, cfg=0, dt=0.025, passes=3, steps=4,
                 desc="tiny: o=4, v=16 per spin, Q=48, beta hole, dt=0.025 au"),
    # the paper's ESCA run: 71 occupied / 649 virtual spin-orbitals in total
    # (an 83 GiB (ae|bf) block: one residual is far beyond the oracle's reach on
    # the host, so its CPU baseline is timed on the formaldehyde-shaped system)
    # one residual evaluation plus one step (one fixed-point pass) at o=71, v=649 per spin,
    # amplitudes seeded N(0, 1e-3); steps and warm-up capped by a time budget (one step is
    # minutes in float64); the CPU baseline is the oracle on the same Hamiltonian restricted
    # to its first few virtual orbitals
    "esca": dict(shape=ESCA, cfg=4, dt=0.01, passes=1, steps=1, large=True, seed_amplitudes=1e-3,
                 cpu_slab_vir=6,
                 desc="ESCA-shaped core hole, o=71, v=649 per spin (beta hole: 71/70 occupied, 649/650 "
                      "virtual), Q=2000, L scaled by (16/v)^(1/2), amplitudes seeded N(0,1e-3), one residual "
                      "evaluation plus one step, dt=0.01 au"),
    # Zn-porphyrin shape (655 orbitals: alpha 95/560, beta 94/561 with the hole), one
    # fixed-point pass per step (two amplitude sets), split-precision contractions
    # (its CPU baseline is timed on the formaldehyde-shaped system: the spin-orbital oracle's
    # integral blocks for all 95 occupied orbitals alone exceed a 64 GiB host)
    "zn": dict(shape=ZN_PORPHYRIN, cfg=5, dt=0.01, passes=1, steps=10, large=True, seed_amplitudes=1e-3,
               cpu_sample="formaldehyde",
               desc="Zn-porphyrin-shaped core hole, o=95, v=560 per spin (beta hole: 95/94 occupied, 560/561 "
                    "virtual), Q=3000, L scaled by (16/v)^(1/2), amplitudes seeded N(0,1e-3), one fixed-point "
                    "pass per step, dt=0.01 au"),
    "esca36": dict(shape=ESCA_PAPER, cfg=3, dt=0.01, passes=2, steps=2, large=True, cpu_sample="formaldehyde",
                   desc="ESCA run of the paper's abstract (71 occupied / 649 virtual spin-orbitals in total): "
                        "o=36, v=324 per spin, Q=2000, L scaled by (16/v)^(1/2), beta hole, dt=0.01 au"),
}


def cpu_baseline(name, eps, chol, flops_per_residual):
    """The oracle as it stands: one residual evaluation of workload ``name`` on the host."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import blocks
    from oracle import ccsd, reference
    try:
        import threadpoolctl
        threads = max(int(x.get("num_threads", 1)) for x in threadpoolctl.threadpool_info()) or 1
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    shape = WORKLOADS[name]["shape"]
    sysm = reference.n_minus_one_reference(eps, chol, shape.o, shape.o, 0, 1, lean=True)
    t1, t2 = blocks.random_spin_orbital_amplitudes(sysm, 17, scale=1e-3)
    ccsd._blocks(sysm)                    # integral blocks are built once per propagation
    t0 = time.perf_counter()
    ccsd.residual(sysm, t1, t2)
    dt = time.perf_counter() - t0
    return {"value": flops_per_residual / dt / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"one residual evaluation R(T) of the {name} workload (o={shape.o}, v={shape.v} per spin, "
                      f"Q={shape.nchol}) at seeded amplitudes (spin-orbital oracle, lean integral blocks): "
                      f"{dt:.2f} s; rate = the GPU path's flop count of that residual / that time"}


def cpu_baseline_slab(eps, chol, shape, k_vir, prec, full_flops):
    """The oracle as it stands on a bounded sample of the large workload: the same Hamiltonian
    (orbital energies and Cholesky vectors) restricted to all occupied and the first k_vir
    virtual orbitals; rate = the GPU path's flop count of that restricted residual / the
    oracle's time, and the full residual's CPU time extrapolated at that rate."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import blocks
    from oracle import ccsd, reference
    from paper_2301_04249_amd import rteom
    try:
        import threadpoolctl
        threads = max(int(x.get("num_threads", 1)) for x in threadpoolctl.threadpool_info()) or 1
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    sel = np.r_[0:shape.o, shape.o:shape.o + k_vir]
    eps_s = np.ascontiguousarray(eps[sel])
    chol_s = np.ascontiguousarray(chol[:, sel][:, :, sel])
    sysm = reference.n_minus_one_reference(eps_s, chol_s, shape.o, shape.o, 0, 1, lean=True)
    t1, t2 = blocks.random_spin_orbital_amplitudes(sysm, 17, scale=1e-3)
    blk = ccsd._blocks(sysm)              # integral blocks are built once per propagation
    t0 = time.perf_counter()
    ccsd.residual(sysm, t1, t2, blk)
    dt = time.perf_counter() - t0
    Q = rteom.Propagator(eps_s, chol_s, shape.o, shape.o, 0, 1, prec=prec, workspace="torch", max_steps=2)
    f = Q.residual_flops()
    Q.close()
    rate = f / dt
    return {"value": rate / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"one residual evaluation R(T) of the workload's Hamiltonian restricted to its {shape.o} "
                      f"occupied and first {k_vir} virtual orbitals per spin (same eps and Cholesky vectors; "
                      f"spin-orbital oracle, lean integral blocks, seeded amplitudes): {dt:.2f} s for "
                      f"{f:.3e} flops of the GPU path's count; the full residual ({full_flops:.3e} flops) "
                      f"would take {full_flops / rate:.3e} s at that rate"}


def run_batch(args, work):
    """Batched workload: all systems advance together, each system's captured step replayed on its own stream (timed
    region 1, the value); then the same systems one after another with direct launches and
    HIP events around the ladder launches (timed region 2: roofline and the sequential time)."""
    import torch
    from paper_2301_04249_amd import rteom
    shapes = batched_shapes(work["batch"], cfg=work["cfg"])
    # Cholesky vectors scaled by (16/v)^(1/2): with the unscaled draw the correlation of
    # these shapes is far beyond a molecule's and the propagation overflows within tens
    # of steps (same seeds otherwise)
    systems = [draw_system(sh, cfg=work["cfg"], sys_id=k, chol_scale=(16.0 / sh.v) ** 0.5)
               for k, sh in enumerate(shapes)]
    dt, passes = work["dt"], work["passes"]
    print(f"[bench] workload batched: {len(shapes)} systems", file=sys.stderr, flush=True)

    def props(graph):
        out = []
        for sh, (eps, chol) in zip(shapes, systems):
            out.append(rteom.Propagator(eps, chol, sh.o, sh.o, 0, 1, prec=args.prec, fixed_iters=passes,
                                        fp_map=work.get("fp_map", 0), workspace="torch",
                                        max_steps=args.steps + args.warmup + 4, graph=graph))
        return out

    ps = props(True)
    flops_res = [p.residual_flops() for p in ps]
    B = rteom.Batch(ps)
    print("[bench] batch ready", file=sys.stderr, flush=True)
    if args.warmup:
        B.step(dt, args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    B.step(dt, args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print(f"[bench] batched: {(t1 - t0) * 1e3 / args.steps:.2f} ms/step", file=sys.stderr, flush=True)
    for p in ps:
        if not np.all(np.isfinite(p.cumulant()[1])):
            print("bench.py: non-finite C(t)", file=sys.stderr)
            return 3
    B.close()
    for p in ps:
        p.close()
    del B, ps
    # region 2: sequential, direct launches, ladder timed
    qs = props(False)
    for q in qs:
        q.profile(("ladder",))
        if args.warmup:
            q.step(dt, args.warmup)
    torch.cuda.synchronize()
    for q in qs:
        for ph in rteom.PHASES:
            q.phase_stats(ph)
    torch.cuda.synchronize()
    u0 = time.perf_counter()
    for q in qs:
        q.step(dt, args.steps)
    torch.cuda.synchronize()
    u1 = time.perf_counter()
    lad_ms = lad_flop_total = 0.0
    lad_ops = 0
    for q in qs:
        ms, ops, fl = q.phase_stats("ladder")   # fl: the ladder's flops per residual
        lad_ms += ms
        lad_ops += ops
        lad_flop_total += fl * passes * args.steps
    for q in qs:
        q.close()
    del qs
    n_res = passes * args.steps
    total = sum(flops_res) * n_res
    value = total / (t1 - t0) / 1e12
    useful = lad_flop_total / (lad_ms * 1e-3) / 1e12 if lad_ms > 0 else 0.0
    achieved = useful * EXEC_PER_USEFUL[args.prec]
    peak = PEAK_TFLOPS[args.prec]
    out = {
        "metric": "residual TFLOP/s (time step of the RT-EOM-CCSD hot path)",
        "value": round(value, 4), "unit": "TFLOP/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round((t1 - t0) * 1e3 / args.steps, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE[args.prec],
        "data": "synthetic (seeded eps and Cholesky vectors of the stated shapes)",
        "config": {"workload": work["desc"], "systems": [[sh.o, sh.v, sh.nchol] for sh in shapes],
                   "passes_per_step": passes, "residuals_timed": n_res * len(shapes),
                   "launch": "graph (every system's captured step replayed on its own stream, all systems before any wait)",
                   "flops_per_step": sum(flops_res) * passes,
                   "ms_per_step_sequential_direct": round((u1 - u0) * 1e3 / args.steps, 4),
                   "speedup_vs_sequential_direct": round((u1 - u0) / (t1 - t0), 4)},
        "roofline": {"kernel": KERNEL_NAME[args.prec] + " particle-particle ladders of all systems",
                     "bound": "mfma", "achieved": round(achieved, 4), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 5), "useful_tflops": round(useful, 4),
                     "traffic": TRAFFIC.get(("batched", args.prec)),
                     "launches": lad_ops, "flops_per_launch": lad_flop_total / lad_ops if lad_ops else None,
                     "timing": "HIP events around each ladder launch in a second timed region: the same systems "
                               "and steps one after another with direct launches"},
    }
    if not args.no_cpu_baseline:
        name = work["cpu_sample"]
        sw = WORKLOADS[name]
        eps, chol = draw_system(sw["shape"], cfg=sw["cfg"], chol_scale=chol_scale(sw["shape"]))
        Q = rteom.Propagator(eps, chol, sw["shape"].o, sw["shape"].o, 0, 1, prec=args.prec,
                             fixed_iters=sw["passes"], workspace="torch", max_steps=2)
        f = Q.residual_flops()
        Q.close()
        out["cpu_baseline"] = cpu_baseline(name, eps, chol, f)
    print(json.dumps(out), flush=True)
    return 0


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default: per workload)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="esca", choices=sorted(WORKLOADS))
    ap.add_argument("--budget", type=float, default=330.0,
                    help="seconds for warm-up plus timed steps of the large workloads (caps both)")
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16x3", "fp16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tune", action="store_true",
                    help="time the GEMM tile shapes of every new product (default for the small workloads)")
    ap.add_argument("--tile-cache", default=None, metavar="PATH",
                    help="load timed tile choices from PATH if it exists; with --tune, save them there afterwards")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run a device-to-device copy of BYTES (HBM counter calibration) and exit")
    args = ap.parse_args(argv)
    if args.copy_probe:
        import torch
        n = args.copy_probe // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": n * 8}))
        return 0
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the benchmark runs on one GPU (the hot path of one propagation per GPU); run with --gpus 1",
              file=sys.stderr)
        return 2

    import torch
    from paper_2301_04249_amd import rteom

    torch.cuda.set_device(0)
    work = WORKLOADS[args.workload]
    if args.steps is None:
        args.steps = work["steps"]
    if work.get("batch"):
        return run_batch(args, work)
    shape = work["shape"]
    scale = chol_scale(shape) if shape.v > 16 else 1.0
    eps, chol = draw_system(shape, cfg=work["cfg"], chol_scale=scale)
    print(f"[bench] workload {args.workload}: {work['desc']}", file=sys.stderr, flush=True)
    dt = work["dt"]
    large = bool(work.get("large"))
    req_steps, req_warmup = args.steps, args.warmup

    def run(graph):
        P = rteom.Propagator(eps, chol, shape.o, shape.o, 0, 1, prec=args.prec, fixed_iters=work["passes"],
                             workspace="torch", max_steps=req_steps + req_warmup + 4, graph=graph,
                             tune=args.tune or not large, progress=large)
        if args.tile_cache and os.path.exists(args.tile_cache):
            P.load_tiles(args.tile_cache)
        plan = P.plan()
        print(f"[bench] {'graph' if graph else 'direct'} launches: context ready, plan {plan}", file=sys.stderr,
              flush=True)
        steps, warmup = req_steps, req_warmup
        if large:
            # one step is minutes: warm-up and timed steps within the time budget, at a
            # conservative rate estimate (no warm-up is needed for timing: the kernels are
            # compiled ahead and the tile shapes come from the rule, not from timing)
            t_est = work["passes"] * P.residual_flops() / (RATE_GUESS[args.prec] * 1e12)
            warmup = int(min(req_warmup, max(0.0, args.budget - t_est) // t_est))
            steps = int(max(1, min(req_steps, (args.budget - warmup * t_est) // t_est)))
            print(f"[bench] estimated {t_est:.0f} s per step: {warmup} warm-up and {steps} timed step(s) "
                  f"in the {args.budget:.0f} s budget", file=sys.stderr, flush=True)
        if work.get("seed_amplitudes"):
            # amplitudes drawn N(0, sigma^2) (real and imaginary parts) on the device, in place
            x, _ = P.device_sets()
            gen = torch.Generator(device="cuda")
            gen.manual_seed(23014249)
            chunk = 1 << 26
            for k in range(0, x.numel(), chunk):
                m = min(chunk, x.numel() - k)
                x[k:k + m] = torch.randn(m, generator=gen, device="cuda", dtype=torch.float64) * work["seed_amplitudes"]
            P.amplitudes_written()
            torch.cuda.synchronize()
        if not graph:
            P.profile(rteom.PHASES if large else ("ladder",))   # HIP events on the engine stream
        if warmup:
            P.step(dt, warmup)       # raises NONFINITE if the amplitudes overflowed
        torch.cuda.synchronize()
        print(f"[bench] warmup done ({warmup} steps)", file=sys.stderr, flush=True)
        for ph in rteom.PHASES:
            P.phase_stats(ph)             # clear
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters = P.step(dt, steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        print(f"[bench] timed {steps} steps: {(t1 - t0) * 1e3 / steps:.2f} ms/step", file=sys.stderr, flush=True)
        stats = {ph: P.phase_stats(ph) for ph in rteom.PHASES}
        if args.tune and args.tile_cache:
            P.save_tiles(args.tile_cache)
        return P, iters, t0, t1, stats, steps, warmup

    # Timed region 1 gives the value.  Small workloads replay each step as a
    # hipGraph (launch overhead matters there); large ones launch directly, with
    # HIP events around every operation in the same region.
    mode = "direct" if large else "graph"
    if mode == "graph":
        try:
            P, iters, t0, t1, _, steps, warmup = run(True)
        except rteom.RteomError as exc:    # graph capture unavailable: launch operations directly
            print(f"[bench] graph mode failed ({exc}); direct launches", file=sys.stderr, flush=True)
            mode = "direct"
    ms_direct = None
    if mode == "graph":
        # Timed region 2 (roofline only): the same steps with direct launches and
        # HIP events around every ladder launch; events cannot time kernels inside
        # a replayed graph.
        P2, _, u0, u1, stats, _, _ = run(False)
        ms_direct = (u1 - u0) * 1e3 / steps
        P2.close()
    else:
        P, iters, t0, t1, stats, steps, warmup = run(False)
    lad_ms, lad_ops, lad_flops = stats["ladder"]
    flops_res = P.residual_flops()
    plan = P.plan()
    n_res = int(np.sum(iters))
    ms_per_step = (t1 - t0) * 1e3 / steps
    value = flops_res * n_res / (t1 - t0) / 1e12
    _, c = P.cumulant()
    if not np.all(np.isfinite(c)):
        print("bench.py: non-finite C(t)", file=sys.stderr)
        return 3
    # the ladder phase: its launches are the dominant kernel's (alpha-beta block in full
    # storage, both same-spin blocks in pair storage; per integral slab when not resident)
    lad_total = lad_flops * n_res
    useful = lad_total / (lad_ms * 1e-3) / 1e12 if lad_ms > 0 else 0.0
    achieved = useful * EXEC_PER_USEFUL[args.prec]   # executed matrix-core flops
    avg_ms = lad_ms / lad_ops if lad_ops else None
    traffic = TRAFFIC.get((args.workload, args.prec))
    peak = PEAK_TFLOPS[args.prec]
    launch = {"graph": "graph (each time step captured once as a hipGraph and replayed)",
              "direct": "direct (every operation launched on one HIP stream)"}[mode]
    config = {"workload": work["desc"], "chol_scale": scale, "passes_per_step": work["passes"],
              "residuals_timed": n_res, "steps_requested": req_steps, "warmup_requested": req_warmup,
              "launch": launch, "flops_per_residual": flops_res, "exec_flops_per_residual": plan["exec_flops"],
              "s_per_residual": (t1 - t0) / n_res, "memory_plan": plan,
              "tile_choice": ("timed" if args.tune or not large else "rule")
                             + (f", cache {args.tile_cache}" if args.tile_cache else "")}
    if ms_direct is not None:
        config["ms_per_step_direct_launch"] = round(ms_direct, 4)
    if large:
        config["phases_s_per_residual"] = {ph: round(v[0] / 1e3 / n_res, 4) for ph, v in stats.items()}
        config["phases_tflops"] = {ph: round(v[2] * n_res / (v[0] * 1e-3) / 1e12, 3)
                                   for ph, v in stats.items() if v[0] > 0 and v[2] > 0}
    out = {
        "metric": "residual TFLOP/s (time step of the RT-EOM-CCSD hot path)",
        "value": round(value, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.prec],
        "data": "synthetic (seeded eps, Cholesky vectors" + (" and amplitudes" if work.get("seed_amplitudes") else "")
                + " of the stated shape)",
        "config": config,
        "roofline": {"kernel": KERNEL_NAME[args.prec] + " particle-particle ladder (alpha-beta block in full "
                               "storage, both same-spin blocks in pair storage)",
                     "bound": "mfma", "achieved": round(achieved, 4), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 5), "useful_tflops": round(useful, 4),
                     "traffic": traffic[0] if traffic else None,
                     "traffic_source": traffic[1] if traffic else None,
                     "launches": lad_ops, "flops_per_launch": lad_total / lad_ops if lad_ops else None,
                     "avg_launch_ms": round(avg_ms, 5) if avg_ms else None,
                     "timing": "HIP events on the engine stream around each ladder launch, " + (
                         "in a second timed region of the same steps with direct launches" if mode == "graph"
                         else "in the timed region")},
    }
    if not args.no_cpu_baseline:
        if work.get("cpu_slab_vir"):
            P.close()
            del P
            torch.cuda.empty_cache()
            out["cpu_baseline"] = cpu_baseline_slab(eps, chol, shape, work["cpu_slab_vir"], args.prec, flops_res)
        else:
            name = work.get("cpu_sample", args.workload)
            if name != args.workload:
                P.close()
                del P
                sw = WORKLOADS[name]
                eps, chol = draw_system(sw["shape"], cfg=sw["cfg"], chol_scale=chol_scale(sw["shape"]))
                Q = rteom.Propagator(eps, chol, sw["shape"].o, sw["shape"].o, 0, 1, prec=args.prec,
                                     fixed_iters=sw["passes"], workspace="torch", max_steps=2)
                flops_res = Q.residual_flops()
                Q.close()
            out["cpu_baseline"] = cpu_baseline(name, eps, chol, flops_res)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
