"""Ground-state CCSD of the N-electron reference (test infrastructure, CPU, float64).

The cumulant Green's function carries the phase of the N-electron ground state,
E_N = E_N^HF + E_N^corr (Sec. 2.2, Eqs. cum_gf and cum_gf2); the paper takes E_N^corr from a
ground-state CCSD calculation.  That is the stationary point of the same amplitude equations:
R(T) = <Phi_x|e^{-T} H_N e^{T}|Phi> = 0 for the N-electron determinant, with
E_N^corr = <Phi|(H_N e^T)_C|Phi> at the solution (Eq. cum_gf3's integrand).

The solver is the textbook Jacobi iteration on R = RHS - D*t: t <- t + R / D, with the
orbital-energy denominators D of ccsd.residual, from t = 0 until max |change| < tol.
MP2 (the first step of that iteration from t = 0, as an energy) is the weak-coupling limit.
"""
from __future__ import annotations

import numpy as np

from . import ccsd
from .propagate import _denominators
from .reference import SpinOrbitalSystem


class NoConvergence(RuntimeError):
    pass


def solve(sys: SpinOrbitalSystem, tol: float = 1e-10, max_iter: int = 200):
    """(E_corr, t1, t2, iterations) of the ground-state CCSD equations by Jacobi iteration."""
    d1, d2 = _denominators(sys)
    t1, t2 = ccsd.zero_amplitudes(sys)
    mask1, mask2 = d1 != 0, d2 != 0
    for it in range(1, max_iter + 1):
        r1, r2 = ccsd.residual(sys, t1, t2)
        n1 = np.where(mask1, t1 + r1 / np.where(mask1, d1, 1.0), 0.0)
        n2 = np.where(mask2, t2 + r2 / np.where(mask2, d2, 1.0), 0.0)
        change = max(np.abs(n1 - t1).max(initial=0.0), np.abs(n2 - t2).max(initial=0.0))
        t1, t2 = n1, n2
        if change < tol:
            return ccsd.energy(sys, t1, t2), t1, t2, it
    raise NoConvergence(f"ground-state CCSD not converged in {max_iter} iterations")


def mp2_energy(sys: SpinOrbitalSystem) -> float:
    """Second-order (MP2) correlation energy for a canonical reference:
    1/4 sum |<ij||ab>|^2 / (f_ii + f_jj - f_aa - f_bb)."""
    _, d2 = _denominators(sys)
    v = sys.block("oovv")
    return float(0.25 * np.sum(v * v / d2))
