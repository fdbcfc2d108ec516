"""Spin-orbital (N-1)-electron reference for the RT-EOM-CC core-hole problem.

Paper, Sec. 2.1 (after Eq. amp): the reference |Phi> is the N-electron
Hartree-Fock determinant with the core spin-orbital c annihilated; c joins the
unoccupied set.  The Hamiltonian is normal ordered with respect to |Phi>, with
Fock elements f_pq = eps_p delta_pq - <pc||qc>.  Sec. 2.3: the two-electron
integrals are Cholesky factorised, (pq|rs) = sum_Q L^Q_pq L^Q_rs.

Spin-orbital index convention used throughout the oracle: spin-orbital
``p + n * s`` is spatial orbital p with spin s (0 = alpha, 1 = beta).
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class SpinOrbitalSystem:
    n: int                    # spatial orbitals
    eps: np.ndarray           # [n] N-electron orbital energies
    chol: np.ndarray          # [Q, n, n]
    occ: np.ndarray           # spin-orbital indices occupied in Phi
    vir: np.ndarray           # spin-orbital indices unoccupied in Phi
    core: int                 # spin-orbital index of c
    fock: np.ndarray          # [2n, 2n] f_pq of the (N-1) reference
    g: np.ndarray             # [2n, 2n, 2n, 2n] <pq||rs>

    @property
    def nso(self) -> int:
        return 2 * self.n

    @property
    def no(self) -> int:
        return len(self.occ)

    @property
    def nv(self) -> int:
        return len(self.vir)

    def block(self, spec: str) -> np.ndarray:
        """Sub-block of <pq||rs> with 'o'/'v' per index, e.g. 'oovv'."""
        idx = [self.occ if c == "o" else self.vir for c in spec]
        return self.g[np.ix_(*idx)]

    def fblock(self, spec: str) -> np.ndarray:
        idx = [self.occ if c == "o" else self.vir for c in spec]
        return self.fock[np.ix_(*idx)]


def coulomb_from_cholesky(chol: np.ndarray) -> np.ndarray:
    """Spatial chemists'-notation integrals (pq|rs) = sum_Q L^Q_pq L^Q_rs (Sec. 2.3)."""
    nq, n, _ = chol.shape
    lf = chol.reshape(nq, n * n)
    return (lf.T @ lf).reshape(n, n, n, n)


def antisymmetrized_spin_orbital(eri: np.ndarray) -> np.ndarray:
    """<pq||rs> = <pq|rs> - <pq|sr> with <pq|rs> = (pr|qs) delta(sp,sr) delta(sq,ss)."""
    n = eri.shape[0]
    nso = 2 * n
    spin = np.repeat([0, 1], n)
    sp = np.tile(np.arange(n), 2)
    # physicists' <pq|rs> over spin-orbitals
    phys = eri[np.ix_(sp, sp, sp, sp)].transpose(0, 2, 1, 3)  # (pr|qs) -> [p,q,r,s]
    same_pr = spin[:, None] == spin[None, :]
    mask = same_pr[:, None, :, None] & same_pr[None, :, None, :]  # [p,q,r,s]: sp==sr, sq==ss
    phys = np.where(mask, phys, 0.0)
    return phys - phys.transpose(0, 1, 3, 2)


def n_minus_one_reference(eps, chol, n_occ_a: int, n_occ_b: int, core_orb: int,
                          core_spin: int) -> SpinOrbitalSystem:
    """Build the (N-1)-electron reference by removing spin-orbital (core_orb, core_spin).

    The N-electron determinant occupies spatial orbitals 0..n_occ_s-1 in spin s.
    """
    eps = np.asarray(eps, dtype=np.float64)
    chol = np.asarray(chol, dtype=np.float64)
    n = eps.shape[0]
    occ_n = [p for p in range(n_occ_a)] + [p + n for p in range(n_occ_b)]
    core = core_orb + n * core_spin
    if core not in occ_n:
        raise ValueError("core spin-orbital is not occupied in the N-electron reference")
    occ = np.array(sorted(set(occ_n) - {core}), dtype=np.int64)
    vir = np.array(sorted(set(range(2 * n)) - set(occ.tolist())), dtype=np.int64)
    eri = coulomb_from_cholesky(chol)
    g = antisymmetrized_spin_orbital(eri)
    eps_so = np.concatenate([eps, eps])
    # f_pq = eps_p delta_pq - <pc||qc>  (the Fock definition beside the normal-ordered H_N)
    fock = np.diag(eps_so) - g[:, core, :, core]
    return SpinOrbitalSystem(n=n, eps=eps, chol=chol, occ=occ, vir=vir, core=core,
                             fock=fock, g=g)


def one_body_core(sys: SpinOrbitalSystem) -> np.ndarray:
    """h_pq implied by the Fock matrix of Phi: h = f - sum_{k in occ(Phi)} <pk||qk>."""
    return sys.fock - np.einsum("pkqk->pq", sys.g[:, sys.occ][:, :, :, sys.occ])
