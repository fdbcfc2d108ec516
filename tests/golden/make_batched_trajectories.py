"""Write the oracle's short trajectories of the batched workload's members.

Calls only ``oracle/`` (and the seeded draws of ``synthetic/``).  The batched workload
is 16 independent core holes of uneven shape (o in [5,20], v in [40,200] per spin,
Q = 4v; seeds cfg=2, sys=k), Cholesky vectors scaled by (16/v)^(1/2), the diagonal
("denominator") fixed-point map with exactly PASSES passes per step, dt = DT, STEPS
steps from T(0) = 0, C(t) by Eq. cum_gf3.  Members whose spin-orbital integral blocks
do not fit the host memory of the machine that writes the file (v above VMAX) are left
out; the file lists the members it holds.

    python tests/golden/make_batched_trajectories.py

Output: tests/golden/batched_trajectories.txt, one line per (member, time point):
member o v Q t Re C Im C.
"""
from __future__ import annotations

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import propagate, reference  # noqa: E402
from synthetic import batched_shapes, draw_system  # noqa: E402

DT = 0.025
PASSES = 2
STEPS = 3
CFG = 2
VMAX = 125
OUT = os.path.join(HERE, "batched_trajectories.txt")


def main():
    shapes = batched_shapes(16, cfg=CFG)
    lines = []
    for k, sh in enumerate(shapes):
        if sh.v > VMAX:
            print(f"member {k} {sh}: left out (v > {VMAX})", flush=True)
            continue
        t0 = time.time()
        eps, chol = draw_system(sh, cfg=CFG, sys_id=k, chol_scale=(16.0 / sh.v) ** 0.5)
        sysm = reference.n_minus_one_reference(eps, chol, sh.o, sh.o, 0, 1, lean=True)
        tr = propagate.propagate(sysm, DT, STEPS, fixed_iters=PASSES, fp_map="denominator")
        for t, c in zip(tr.times, tr.cumulant):
            lines.append(f"{k} {sh.o} {sh.v} {sh.nchol} {t:.6f} {c.real:.17e} {c.imag:.17e}\n")
        print(f"member {k} {sh}: C(t_n) = {tr.cumulant[-1]:.12e} ({time.time() - t0:.0f} s)", flush=True)
        del sysm, tr
    with open(OUT, "w") as f:
        f.write("# Oracle trajectories of the batched workload's members "
                "(tests/golden/make_batched_trajectories.py):\n")
        f.write(f"# L scaled by (16/v)^(1/2), diagonal fixed-point map, {PASSES} passes per step, dt={DT}, "
                f"{STEPS} steps, seeds cfg={CFG} sys=member; members with v > {VMAX} left out.\n")
        f.write("# member o v Q t re_C im_C\n")
        f.writelines(lines)
    print(f"wrote {OUT}")


if __name__ == "__main__":
    main()
