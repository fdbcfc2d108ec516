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

from synthetic import FORMALDEHYDE, TINY, draw_system  # noqa: E402

# MI355X published peaks (dense)
PEAK_TFLOPS = {"fp64": 78.6, "fp32": 157.3, "bf16x3": 2500.0}
PEAK_HBM_GBS = 8000.0

WORKLOADS = {
    "formaldehyde": dict(shape=FORMALDEHYDE, cfg=1, dt=0.025, passes=3,
                         desc="formaldehyde-shaped core hole: o=8, v=110 per spin, Q=600, beta hole, dt=0.025 au"),
    "tiny": dict(shape=TINY, cfg=0, dt=0.025, passes=3,
                 desc="tiny: o=4, v=16 per spin, Q=48, beta hole, dt=0.025 au"),
}


def cpu_baseline(work, eps, chol, flops_per_residual):
    """The oracle as it stands: one residual evaluation of the same workload on the host."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import blocks
    from oracle import ccsd, reference
    try:
        import threadpoolctl
        threads = max(int(x.get("num_threads", 1)) for x in threadpoolctl.threadpool_info()) or 1
    except Exception:  # pragma: no cover
        threads = os.cpu_count() or 1
    shape = work["shape"]
    sysm = reference.n_minus_one_reference(eps, chol, shape.o, shape.o, 0, 1, lean=True)
    t1, t2 = blocks.random_spin_orbital_amplitudes(sysm, 17, scale=1e-3)
    ccsd._blocks(sysm)                    # integral blocks are built once per propagation
    t0 = time.perf_counter()
    ccsd.residual(sysm, t1, t2)
    dt = time.perf_counter() - t0
    return {"value": flops_per_residual / dt / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
            "sample": f"one residual evaluation R(T) of the {shape.o}/{shape.v}/Q={shape.nchol} workload at seeded "
                      f"amplitudes (spin-orbital oracle, lean integral blocks): {dt:.2f} s; rate = the GPU path's "
                      f"flop count of one residual / that time"}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="formaldehyde", choices=sorted(WORKLOADS))
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
        print("bench.py: this build measures one GPU only (single-GPU hot path); run with --gpus 1",
              file=sys.stderr)
        return 2

    import torch
    from paper_2301_04249_amd import rteom

    torch.cuda.set_device(0)
    work = WORKLOADS[args.workload]
    shape = work["shape"]
    eps, chol = draw_system(shape, cfg=work["cfg"])
    print(f"[bench] workload {args.workload}: {work['desc']}", file=sys.stderr, flush=True)
    dt = work["dt"]

    def run(graph):
        P = rteom.Propagator(eps, chol, shape.o, shape.o, 0, 1, prec=args.prec, fixed_iters=work["passes"],
                             workspace="torch", max_steps=args.steps + args.warmup + 4, graph=graph)
        # HIP events around the dominant kernel only; in graph mode they are event
        # nodes of the captured step, re-recorded by every replay
        P.profile(("ladder",))
        if args.warmup:
            P.step(dt, args.warmup)
        torch.cuda.synchronize()
        for ph in rteom.PHASES:
            P.phase_stats(ph)             # clear
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters = P.step(dt, args.steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        stats = P.phase_stats("ladder")
        return P, iters, t0, t1, stats

    mode = "graph"
    try:
        P, iters, t0, t1, (lad_ms, lad_ops, lad_flops) = run(True)
    except rteom.RteomError as exc:    # graph capture unavailable: launch operations directly
        print(f"[bench] graph mode failed ({exc}); direct launches", file=sys.stderr, flush=True)
        mode = "direct"
        P, iters, t0, t1, (lad_ms, lad_ops, lad_flops) = run(False)
    P.profile(())
    flops_res = P.residual_flops()
    n_res = int(np.sum(iters))
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    value = flops_res * n_res / (t1 - t0) / 1e12
    _, c = P.cumulant()
    if not np.all(np.isfinite(c)):
        print("bench.py: non-finite C(t)", file=sys.stderr)
        return 3
    achieved = lad_flops * lad_ops / (lad_ms * 1e-3) / 1e12 if lad_ms > 0 else 0.0
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
        "dtype": {"fp64": "f64", "fp32": "f32 contractions, f64 update", "bf16x3": "bf16x3 contractions (f32 accumulate), f64 update"}[args.prec],
        "data": "synthetic (seeded eps and Cholesky vectors of the stated shape)",
        "config": {"workload": work["desc"], "passes_per_step": work["passes"], "residuals_timed": n_res,
                   "launch": mode + (" (each time step captured once as a hipGraph and replayed)" if mode == "graph" else ""),
                   "flops_per_residual": flops_res, "s_per_residual": (t1 - t0) / n_res},
        "roofline": {"kernel": "gemm_f64 particle-particle ladder (3 spin blocks in one launch)",
                     "bound": "mfma", "achieved": round(achieved, 4), "peak": PEAK_TFLOPS[args.prec],
                     "unit": "TFLOP/s", "frac": round(achieved / PEAK_TFLOPS[args.prec], 5), "traffic": None,
                     "launches": lad_ops, "flops_per_launch": lad_flops,
                     "timing": "HIP events around the ladder launches" + (
                         " (event nodes of the step graph: the launches of the last timed step)" if mode == "graph"
                         else " in the timed region"),
                     "avg_launch_ms": (lad_ms / lad_ops) if lad_ops else None},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(work, eps, chol, flops_res)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
