"""Test helpers: map between the oracle's spin-orbital amplitudes and the
library's extended spin-blocked layout (include/rteom.h), and build seeded
amplitudes.  Index bookkeeping only; no arithmetic of the method.
"""
import numpy as np


def index_maps(sys, occ_list, vir_list):
    """For spin s: arrays (i_ext -> oracle occ index or -1), (a_ext -> oracle vir index or -1)."""
    n = sys.n
    occ = {int(p): k for k, p in enumerate(sys.occ)}
    vir = {int(p): k for k, p in enumerate(sys.vir)}
    om, vm = [], []
    for s in (0, 1):
        om.append(np.array([occ.get(int(p) + n * s, -1) for p in occ_list]))
        vm.append(np.array([vir.get(int(p) + n * s, -1) for p in vir_list]))
    return om, vm


def to_blocks(sys, occ_list, vir_list, t1, t2):
    """Spin-orbital (t1[i,a], t2[i,j,a,b]) -> (t1[2,no,nv], t2[3,no,no,nv,nv])."""
    om, vm = index_maps(sys, occ_list, vir_list)
    no, nv = len(occ_list), len(vir_list)
    b1 = np.zeros((2, no, nv), dtype=complex)
    for s in (0, 1):
        oi, vi = om[s], vm[s]
        ok = (oi[:, None] >= 0) & (vi[None, :] >= 0)
        b1[s] = np.where(ok, t1[np.ix_(np.maximum(oi, 0), np.maximum(vi, 0))], 0)
    b2 = np.zeros((3, no, no, nv, nv), dtype=complex)
    for k, (s1, s2) in enumerate(((0, 0), (0, 1), (1, 1))):
        o1, o2, v1, v2 = om[s1], om[s2], vm[s1], vm[s2]
        ok = ((o1[:, None, None, None] >= 0) & (o2[None, :, None, None] >= 0)
              & (v1[None, None, :, None] >= 0) & (v2[None, None, None, :] >= 0))
        vals = t2[np.ix_(np.maximum(o1, 0), np.maximum(o2, 0), np.maximum(v1, 0), np.maximum(v2, 0))]
        b2[k] = np.where(ok, vals, 0)
    return b1, b2


def random_spin_orbital_amplitudes(sys, seed, scale=0.1):
    """Complex Gaussian amplitudes with T2 antisymmetric and spin-forbidden entries zero."""
    rng = np.random.default_rng(seed)
    no, nv = sys.no, sys.nv
    t1 = (rng.standard_normal((no, nv)) + 1j * rng.standard_normal((no, nv))) * scale
    t2 = (rng.standard_normal((no, no, nv, nv)) + 1j * rng.standard_normal((no, no, nv, nv))) * scale
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    so, sv = sys.occ // sys.n, sys.vir // sys.n
    t1 = t1 * (so[:, None] == sv[None, :])
    same = (((so[:, None, None, None] == sv[None, None, :, None]) & (so[None, :, None, None] == sv[None, None, None, :]))
            | ((so[:, None, None, None] == sv[None, None, None, :]) & (so[None, :, None, None] == sv[None, None, :, None])))
    return t1, t2 * same


def random_block_amplitudes(no, nv, seed, scale=1e-3):
    """Seeded blocked amplitudes with antisymmetric aa/bb blocks (for large shapes)."""
    rng = np.random.default_rng(seed)
    t1 = (rng.standard_normal((2, no, nv)) + 1j * rng.standard_normal((2, no, nv))) * scale
    t2 = (rng.standard_normal((3, no, no, nv, nv)) + 1j * rng.standard_normal((3, no, no, nv, nv))) * scale
    for k in (0, 2):
        x = t2[k]
        x = 0.5 * (x - x.transpose(1, 0, 2, 3))
        x = 0.5 * (x - x.transpose(0, 1, 3, 2))
        t2[k] = x
    return t1, t2
