"""Write the oracle's reference trajectory of the formaldehyde-shaped core hole.

Calls only ``oracle/`` (and the seeded draws of ``synthetic/``): the expected
values of the long-propagation parity tests come from here, never from the
library.  The system is the formaldehyde-shaped workload (o=8, v=110 per spin,
Q=600, beta core hole at orbital 0; seeds cfg=1, sys=0) with the Cholesky
vectors scaled by (16/v)^(1/2) -- the literal draw makes the correlation of
this shape far larger than a molecule's and the fixed point of Eq. trapzrule
diverges there.  The trajectory is the implicit trapezoid (Eq. trapzrule) with
exactly PASSES fixed-point passes per step from T(0) = 0, dt = DT, STEPS steps,
C(t) by the same trapezoid weights (Eq. cum_gf3), then A(omega) and its
quasi-particle peak (Eqs. cum_gf, cum_gf2) on OMEGAS with damping ETA.

    python tests/golden/make_formaldehyde_trajectory.py [--steps N] [--fp-map denominator --out FILE]

Output: tests/golden/formaldehyde_trajectory.txt (one line per time point:
t, Re C, Im C, Re E, Im E; header lines start with '#').  One oracle residual
takes ~17 s on 8 host cores, so the default run takes about two hours.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import ccsd, propagate, reference  # noqa: E402
from synthetic import FORMALDEHYDE, draw_system  # noqa: E402

DT = 0.025
PASSES = 2
STEPS = 200
CFG = 1
OMEGA_LO, OMEGA_HI, OMEGA_STEP = -26.0, -14.0, 0.001
ETA = 0.01
OUT = os.path.join(HERE, "formaldehyde_trajectory.txt")


def chol_scale(v: int) -> float:
    return (16.0 / v) ** 0.5


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=STEPS)
    ap.add_argument("--out", default=OUT)
    ap.add_argument("--fp-map", default="plain", choices=["plain", "denominator"],
                    help="fixed-point map of the passes (denominator: the diagonal part taken implicitly)")
    args = ap.parse_args(argv)
    sh = FORMALDEHYDE
    eps, chol = draw_system(sh, cfg=CFG, chol_scale=chol_scale(sh.v))
    sysm = reference.n_minus_one_reference(eps, chol, sh.o, sh.o, 0, 1, lean=True)
    blocks = ccsd._blocks(sysm)
    t1, t2 = ccsd.zero_amplitudes(sysm)
    n = args.steps
    times = DT * np.arange(n + 1)
    cum = np.zeros(n + 1, dtype=complex)
    ens = np.zeros(n + 1, dtype=complex)
    ens[0] = ccsd.energy(sysm, t1, t2)
    t0 = time.time()
    for k in range(n):
        t1, t2, _ = propagate.trapezoid_step(sysm, t1, t2, DT, fixed_iters=PASSES, fp_map=args.fp_map, blocks=blocks)
        ens[k + 1] = ccsd.energy(sysm, t1, t2)
        cum[k + 1] = cum[k] + 0.5j * DT * (ens[k] + ens[k + 1])
        print(f"step {k + 1}/{n}: C = {cum[k + 1]:.12e} ({time.time() - t0:.0f} s)", flush=True)
        if not np.isfinite(cum[k + 1]):
            raise SystemExit("non-finite C(t)")
    omegas = np.arange(OMEGA_LO, OMEGA_HI, OMEGA_STEP)
    g = propagate.green_function(times, cum, eps[0])
    a = propagate.spectral_function(times, g, omegas, ETA)
    qp = propagate.qp_peak(omegas, a)
    with open(args.out, "w") as f:
        f.write("# Oracle trajectory (tests/golden/make_formaldehyde_trajectory.py): formaldehyde-shaped core hole,\n")
        f.write(f"# o={sh.o} v={sh.v} per spin, Q={sh.nchol}, beta hole at orbital 0, seeds cfg={CFG} sys=0,\n")
        f.write(f"# Cholesky vectors scaled by (16/v)^(1/2) = {chol_scale(sh.v):.17g}; Eq. trapzrule with\n")
        f.write(f"# {PASSES} fixed-point passes per step ({args.fp_map} map), dt={DT}, {n} steps; C(t) by Eq. cum_gf3.\n")
        f.write(f"# spectral: omega in [{OMEGA_LO}, {OMEGA_HI}) step {OMEGA_STEP}, eta={ETA}, e_corr=0\n")
        f.write(f"# qp_peak {qp:.15f}\n")
        f.write(f"# a_max {a.max():.15e}\n")
        f.write("# t re_C im_C re_E im_E\n")
        for k in range(n + 1):
            f.write(f"{times[k]:.6f} {cum[k].real:.17e} {cum[k].imag:.17e} {ens[k].real:.17e} {ens[k].imag:.17e}\n")
    print(f"wrote {args.out}: QP peak {qp:.9f} Eh, max |C| {np.abs(cum).max():.4e}")


if __name__ == "__main__":
    main()
