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

from synthetic import ESCA_PAPER, FORMALDEHYDE, TINY, batched_shapes, draw_system  # noqa: E402

# Ladder kernel per precision (the contraction's MFMA instruction family)
KERNEL_NAME = {"fp64": "gemm_mfma<double>", "fp32": "gemm_mfma<float> (operands converted to float planes)",
               "bf16x3": "gemm_bf16x3_split (operands split into bf16 hi/lo planes)"}

# HBM bytes per ladder launch from rocprofv3 --pmc FETCH_SIZE and WRITE_SIZE,
# scaled by the same counters read on a plain device copy of known size; the
# summaries (with the commands) are under profiles/.  Only workloads whose
# ladder kernel has been counted since its last change are listed.
TRAFFIC = {
    # profiles/gemm_mfma_ladder_esca_fp64.md: FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, mean of the
    # alpha-beta and same-spin ladder launches
    ("esca36", "fp64"): 7.94e11,
}

DTYPE = {"fp64": "f64", "fp32": "f32 contractions, f64 update",
         "bf16x3": "bf16x3 contractions (f32 accumulate), f64 update"}

# Matrix-core flops executed per useful flop: the split precision runs three bf16
# products (hi*hi, hi*lo, lo*hi) per product; its roofline counts executed flops
EXEC_PER_USEFUL = {"fp64": 1.0, "fp32": 1.0, "bf16x3": 3.0}

# MI355X published peaks (dense)
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}
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
                         "Q = 4 v, L scaled by (16/v)^(1/2), beta holes), diagonal fixed-point map, one graph "
                         "launch per time step for all, dt=0.025 au"),
    "tiny": dict(shape=TINY, cfg=0, dt=0.025, passes=3, steps=4,
                 desc="tiny: o=4, v=16 per spin, Q=48, beta hole, dt=0.025 au"),
    # the paper's ESCA run: 71 occupied / 649 virtual spin-orbitals in total
    # (an 83 GiB (ae|bf) block: one residual is far beyond the oracle's reach on
    # the host, so its CPU baseline is timed on the formaldehyde-shaped system)
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


def run_batch(args, work):
    """Batched workload: all systems advance together, one graph launch per time step (timed
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
                   "launch": "graph (one launch of a graph holding every system's captured step)",
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
    ap.add_argument("--workload", default="esca36", choices=sorted(WORKLOADS))
    ap.add_argument("--prec", default="fp64", choices=["fp64", "fp32", "bf16x3"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
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

    def run(graph):
        P = rteom.Propagator(eps, chol, shape.o, shape.o, 0, 1, prec=args.prec, fixed_iters=work["passes"],
                             workspace="torch", max_steps=args.steps + args.warmup + 4, graph=graph)
        if not graph:
            P.profile(("ladder",))        # HIP events around the dominant kernel only
        print(f"[bench] {'graph' if graph else 'direct'} launches: context ready", file=sys.stderr, flush=True)
        if args.warmup:
            P.step(dt, args.warmup)       # raises NONFINITE if the amplitudes overflowed
        torch.cuda.synchronize()
        print(f"[bench] warmup done ({args.warmup} steps)", file=sys.stderr, flush=True)
        for ph in rteom.PHASES:
            P.phase_stats(ph)             # clear
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters = P.step(dt, args.steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        print(f"[bench] timed {args.steps} steps: {(t1 - t0) * 1e3 / args.steps:.2f} ms/step", file=sys.stderr,
              flush=True)
        stats = P.phase_stats("ladder")
        return P, iters, t0, t1, stats

    # Timed region 1 gives the value.  Small workloads replay each step as a
    # hipGraph (launch overhead matters there); large ones launch directly, with
    # HIP events around every ladder launch in the same region.
    mode = "direct" if work.get("large") else "graph"
    if mode == "graph":
        try:
            P, iters, t0, t1, _ = run(True)
        except rteom.RteomError as exc:    # graph capture unavailable: launch operations directly
            print(f"[bench] graph mode failed ({exc}); direct launches", file=sys.stderr, flush=True)
            mode = "direct"
    ms_direct = None
    if mode == "graph":
        # Timed region 2 (roofline only): the same steps with direct launches and
        # HIP events around every ladder launch; events cannot time kernels inside
        # a replayed graph.
        P2, _, u0, u1, (lad_ms, lad_ops, lad_flops) = run(False)
        ms_direct = (u1 - u0) * 1e3 / args.steps
        P2.close()
    else:
        P, iters, t0, t1, (lad_ms, lad_ops, lad_flops) = run(False)
    flops_res = P.residual_flops()
    n_res = int(np.sum(iters))
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = flops_res * n_res / (t1 - t0) / 1e12
    _, c = P.cumulant()
    if not np.all(np.isfinite(c)):
        print("bench.py: non-finite C(t)", file=sys.stderr)
        return 3
    # the ladder phase: two launches per residual (alpha-beta block, same-spin pairs)
    lad_total = lad_flops * n_res
    useful = lad_total / (lad_ms * 1e-3) / 1e12 if lad_ms > 0 else 0.0
    achieved = useful * EXEC_PER_USEFUL[args.prec]   # executed matrix-core flops
    avg_ms = lad_ms / lad_ops if lad_ops else None
    traffic = TRAFFIC.get((args.workload, args.prec))
    peak = PEAK_TFLOPS[args.prec]
    launch = {"graph": "graph (each time step captured once as a hipGraph and replayed)",
              "direct": "direct (every operation launched on one HIP stream)"}[mode]
    config = {"workload": work["desc"], "chol_scale": scale, "passes_per_step": work["passes"],
              "residuals_timed": n_res,
              "launch": launch, "flops_per_residual": flops_res, "s_per_residual": (t1 - t0) / n_res}
    if ms_direct is not None:
        config["ms_per_step_direct_launch"] = round(ms_direct, 4)
    out = {
        "metric": "residual TFLOP/s (time step of the RT-EOM-CCSD hot path)",
        "value": round(value, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.prec],
        "data": "synthetic (seeded eps and Cholesky vectors of the stated shape)",
        "config": config,
        "roofline": {"kernel": KERNEL_NAME[args.prec] + " particle-particle ladder (alpha-beta block in full "
                               "storage and both same-spin blocks in pair storage: two launches per residual)",
                     "bound": "mfma", "achieved": round(achieved, 4), "peak": peak, "unit": "TFLOP/s",
                     "frac": round(achieved / peak, 5), "useful_tflops": round(useful, 4),
                     "traffic": traffic,
                     "launches": lad_ops, "flops_per_launch": lad_total / lad_ops if lad_ops else None,
                     "avg_launch_ms": round(avg_ms, 5) if avg_ms else None,
                     "timing": "HIP events on the engine stream around each ladder launch, " + (
                         "in a second timed region of the same steps with direct launches" if mode == "graph"
                         else "in the timed region")},
    }
    if not args.no_cpu_baseline:
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
