"""Brute-force determinant-space evaluation of the RT-EOM-CC projections.

Evaluates the defining expressions directly for tiny systems:

    R_x(T) = <Phi_x| e^{-T} H_N e^{T} |Phi>      (Eqs. dt1eom, dt2eom)
    E(T)   = <Phi| e^{-T} H_N e^{T} |Phi>        (Eq. cum_gf3 integrand)

with H = sum h_pq a+_p a_q + 1/4 sum <pq||rs> a+_p a+_q a_s a_r written as a
dense matrix over all (N-1)-electron determinants, T = T1 + T2 as a matrix,
and e^{+-T} as its finite Taylor series (T is nilpotent on a finite sector).
H_N = H - <Phi|H|Phi>.  Determinants are bit strings over spin-orbitals; the
fermionic sign of a_p is (-1)^(number of occupied spin-orbitals below p).
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from .reference import SpinOrbitalSystem, one_body_core


def _sign_below(det: int, p: int) -> int:
    return -1 if bin(det & ((1 << p) - 1)).count("1") % 2 else 1


def _annihilate(det: int, p: int):
    if not (det >> p) & 1:
        return None, 0
    return det ^ (1 << p), _sign_below(det, p)


def _create(det: int, p: int):
    if (det >> p) & 1:
        return None, 0
    return det | (1 << p), _sign_below(det, p)


def apply_string(det: int, ops):
    """Apply a product of operators right-to-left.  ops: list of ('c'|'a', p), leftmost first."""
    sign = 1
    for kind, p in reversed(ops):
        det, s = (_create if kind == "c" else _annihilate)(det, p)
        if det is None:
            return None, 0
        sign *= s
    return det, sign


class Sector:
    """All determinants with a fixed number of electrons in nso spin-orbitals."""

    def __init__(self, nso: int, nelec: int):
        self.nso = nso
        self.dets = [sum(1 << p for p in c) for c in itertools.combinations(range(nso), nelec)]
        self.index = {d: k for k, d in enumerate(self.dets)}

    @property
    def dim(self):
        return len(self.dets)

    def vector(self, det: int, coeff=1.0):
        v = np.zeros(self.dim, dtype=complex)
        v[self.index[det]] = coeff
        return v


def hamiltonian(sys: SpinOrbitalSystem, sector: Sector) -> np.ndarray:
    h = one_body_core(sys)
    g = sys.g
    nso = sys.nso
    H = np.zeros((sector.dim, sector.dim))
    for col, det in enumerate(sector.dets):
        occ = [p for p in range(nso) if (det >> p) & 1]
        for q in occ:
            for p in range(nso):
                if h[p, q] == 0.0:
                    continue
                d2, s = apply_string(det, [("c", p), ("a", q)])
                if d2 is not None:
                    H[sector.index[d2], col] += s * h[p, q]
        for r, s_ in itertools.permutations(occ, 2):
            d1, sg1 = apply_string(det, [("a", s_), ("a", r)])
            empty = [p for p in range(nso) if not (d1 >> p) & 1]
            for p, q in itertools.permutations(empty, 2):
                val = g[p, q, r, s_]
                if val == 0.0:
                    continue
                d2, sg2 = apply_string(d1, [("c", p), ("c", q)])
                H[sector.index[d2], col] += 0.25 * val * sg1 * sg2
    return H


def reference_det(sys: SpinOrbitalSystem) -> int:
    return sum(1 << int(p) for p in sys.occ)


def cluster_operator(sys: SpinOrbitalSystem, sector: Sector, t1, t2) -> np.ndarray:
    """T = sum_ia t_ia a+_a a_i + sum_{i<j, a<b} t_ijab a+_a a+_b a_j a_i as a matrix."""
    occ, vir = [int(p) for p in sys.occ], [int(p) for p in sys.vir]
    T = np.zeros((sector.dim, sector.dim), dtype=complex)
    singles = [((occ[i], vir[a]), t1[i, a]) for i in range(len(occ)) for a in range(len(vir))]
    doubles = []
    for i, j in itertools.combinations(range(len(occ)), 2):
        for a, b in itertools.combinations(range(len(vir)), 2):
            doubles.append(((occ[i], occ[j], vir[a], vir[b]), t2[i, j, a, b]))
    for col, det in enumerate(sector.dets):
        for (i, a), amp in singles:
            if amp == 0:
                continue
            d2, s = apply_string(det, [("c", a), ("a", i)])
            if d2 is not None:
                T[sector.index[d2], col] += s * amp
        for (i, j, a, b), amp in doubles:
            if amp == 0:
                continue
            d2, s = apply_string(det, [("c", a), ("c", b), ("a", j), ("a", i)])
            if d2 is not None:
                T[sector.index[d2], col] += s * amp
    return T


def _expm_nilpotent(T: np.ndarray, v: np.ndarray, sign: float, max_order: int) -> np.ndarray:
    out = v.copy()
    term = v.copy()
    for k in range(1, max_order + 1):
        term = (sign / k) * (T @ term)
        out = out + term
    return out


def projections(sys: SpinOrbitalSystem, t1, t2):
    """Brute-force (R1, R2, E) for amplitudes (t1, t2); R2 filled for all (i,j,a,b)."""
    nelec = len(sys.occ)
    sector = Sector(sys.nso, nelec)
    H = hamiltonian(sys, sector)
    ref = reference_det(sys)
    phi = sector.vector(ref)
    e_ref = float((phi.conj() @ H @ phi).real)
    HN = H - e_ref * np.eye(sector.dim)
    T = cluster_operator(sys, sector, t1, t2)
    order = nelec + 1
    psi = _expm_nilpotent(T, phi, +1.0, order)
    x = _expm_nilpotent(T, HN @ psi, -1.0, order)
    occ, vir = [int(p) for p in sys.occ], [int(p) for p in sys.vir]
    no, nv = len(occ), len(vir)
    r1 = np.zeros((no, nv), dtype=complex)
    r2 = np.zeros((no, no, nv, nv), dtype=complex)
    for i in range(no):
        for a in range(nv):
            d, s = apply_string(ref, [("c", vir[a]), ("a", occ[i])])
            r1[i, a] = s * x[sector.index[d]]
    for i in range(no):
        for j in range(no):
            if i == j:
                continue
            for a in range(nv):
                for b in range(nv):
                    if a == b:
                        continue
                    d, s = apply_string(ref, [("c", vir[a]), ("c", vir[b]), ("a", occ[j]), ("a", occ[i])])
                    r2[i, j, a, b] = s * x[sector.index[d]]
    energy = complex(x[sector.index[ref]])
    return r1, r2, energy


def exact_overlap(sys: SpinOrbitalSystem, times) -> np.ndarray:
    """<Phi| exp(i H_N tau) |Phi> on a grid, by diagonalising H in the (N-1) sector."""
    nelec = len(sys.occ)
    sector = Sector(sys.nso, nelec)
    H = hamiltonian(sys, sector)
    ref = reference_det(sys)
    k = sector.index[ref]
    e_ref = H[k, k]
    w, U = np.linalg.eigh(H - e_ref * np.eye(sector.dim))
    amp = U[k, :]
    times = np.asarray(times)
    return np.exp(1j * np.outer(times, w)) @ (np.abs(amp) ** 2)


def n_determinants(nso: int, nelec: int) -> int:
    return math.comb(nso, nelec)
