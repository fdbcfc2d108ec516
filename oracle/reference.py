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
    g: object                 # [2n, 2n, 2n, 2n] <pq||rs>, or None (lean: blocks on demand)
    _cache: dict = dataclasses.field(default_factory=dict)

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
        if self.g is not None:
            return self.g[np.ix_(*idx)]
        if spec not in self._cache:
            self._cache[spec] = antisymmetrized_block(self.chol, self.n, *idx)
        return self._cache[spec]

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


def antisymmetrized_block(chol, n, P, Q, R, S):
    """<pq||rs> for spin-orbital index lists P, Q, R, S, built from the Cholesky vectors."""
    P, Q, R, S = (np.asarray(x) for x in (P, Q, R, S))
    sp = lambda x: x % n  # noqa: E731
    ss = lambda x: x // n  # noqa: E731
    # <pq|rs> = (pr|qs) delta(s_p, s_r) delta(s_q, s_s)
    pr = np.einsum("kpr,kqs->pqrs", chol[:, sp(P)][:, :, sp(R)], chol[:, sp(Q)][:, :, sp(S)], optimize=True)
    pr *= (ss(P)[:, None, None, None] == ss(R)[None, None, :, None])
    pr *= (ss(Q)[None, :, None, None] == ss(S)[None, None, None, :])
    # <pq|sr> = (ps|qr) delta(s_p, s_s) delta(s_q, s_r)
    ps = np.einsum("kps,kqr->pqrs", chol[:, sp(P)][:, :, sp(S)], chol[:, sp(Q)][:, :, sp(R)], optimize=True)
    ps *= (ss(P)[:, None, None, None] == ss(S)[None, None, None, :])
    ps *= (ss(Q)[None, :, None, None] == ss(R)[None, None, :, None])
    return pr - ps


def n_minus_one_reference(eps, chol, n_occ_a: int, n_occ_b: int, core_orb: int,
                          core_spin: int, lean: bool = False) -> SpinOrbitalSystem:
    """Build the (N-1)-electron reference by removing spin-orbital (core_orb, core_spin).

    The N-electron determinant occupies spatial orbitals 0..n_occ_s-1 in spin s.
    ``lean=True`` never forms the full (2n)^4 integral tensor: integral blocks are
    built from the Cholesky vectors when first asked for.
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
    eps_so = np.concatenate([eps, eps])
    allso = np.arange(2 * n)
    if lean:
        g = None
        gc = antisymmetrized_block(chol, n, allso, [core], allso, [core])[:, 0, :, 0]
    else:
        g = antisymmetrized_spin_orbital(coulomb_from_cholesky(chol))
        gc = g[:, core, :, core]
    # f_pq = eps_p delta_pq - <pc||qc>  (the Fock definition beside the normal-ordered H_N)
    fock = np.diag(eps_so) - gc
    return SpinOrbitalSystem(n=n, eps=eps, chol=chol, occ=occ, vir=vir, core=core,
                             fock=fock, g=g)


def closed_shell_reference(eps, chol, n_occ_a: int, n_occ_b: int, lean: bool = False) -> SpinOrbitalSystem:
    """The N-electron determinant itself (no ionisation), whose ground-state correlation
    energy E_N^corr enters G(tau) (Sec. 2.2).  The orbital energies are its Fock diagonal:
    f_pq = eps_p delta_pq.  ``core`` is -1."""
    eps = np.asarray(eps, dtype=np.float64)
    chol = np.asarray(chol, dtype=np.float64)
    n = eps.shape[0]
    occ = np.array([p for p in range(n_occ_a)] + [p + n for p in range(n_occ_b)], dtype=np.int64)
    vir = np.array(sorted(set(range(2 * n)) - set(occ.tolist())), dtype=np.int64)
    g = None if lean else antisymmetrized_spin_orbital(coulomb_from_cholesky(chol))
    return SpinOrbitalSystem(n=n, eps=eps, chol=chol, occ=occ, vir=vir, core=-1,
                             fock=np.diag(np.concatenate([eps, eps])), g=g)


def one_body_core(sys: SpinOrbitalSystem) -> np.ndarray:
    """h_pq implied by the Fock matrix of Phi: h = f - sum_{k in occ(Phi)} <pk||qk>."""
    return sys.fock - np.einsum("pkqk->pq", sys.g[:, sys.occ][:, :, :, sys.occ])


def particle_ladder(sys: SpinOrbitalSystem, tau: np.ndarray) -> np.ndarray:
    """1/2 sum_ef <ab||ef> tau_ijef for a tau antisymmetric in (e, f).

    With the full integral tensor this is the plain contraction.  In lean mode the
    antisymmetry of tau turns it into sum_ef (ae|bf) tau_ijef with (ae|bf) the
    spin-orbital Coulomb integral, which connects a with e and b with f of equal
    spin: it is evaluated for each spin of a and of b with the spatial (ae|bf).
    """
    if sys.g is not None:
        return 0.5 * np.einsum("ijef,abef->ijab", tau, sys.block("vvvv"), optimize=True)
    n = sys.n
    vir = sys.vir
    if "ladder" not in sys._cache:
        # constant per system: for each spin pair (sa, sb) the spatial (ae|bf) with a, e
        # of spin sa and b, f of spin sb, as the real matrix [(e, f)][(a, b)]
        spat = np.unique(vir % n)
        pos = {int(p): k for k, p in enumerate(spat)}
        lv = sys.chol[:, spat][:, :, spat]
        vsp = np.einsum("kae,kbf->aebf", lv, lv, optimize=True)   # spatial (ae|bf)
        mats = {}
        for sa in (0, 1):
            A = np.nonzero(vir // n == sa)[0]
            ia = [pos[int(vir[k] % n)] for k in A]
            for sb in (0, 1):
                B = np.nonzero(vir // n == sb)[0]
                ib = [pos[int(vir[k] % n)] for k in B]
                v = vsp[np.ix_(ia, ia, ib, ib)]          # [a, e, b, f]
                mats[sa, sb] = (A, B, np.ascontiguousarray(v.transpose(1, 3, 0, 2)).reshape(
                    len(A) * len(B), len(A) * len(B)))
        del vsp
        sys._cache["ladder"] = mats
    no2 = tau.shape[0] * tau.shape[1]
    out = np.zeros(tau.shape[:2] + (len(vir), len(vir)), dtype=complex)
    for (A, B, m) in sys._cache["ladder"].values():
        # out_ijab = sum_ef tau_ijef (ae|bf) for this spin pair: a real matrix product on the
        # real and the imaginary part of tau
        t = np.ascontiguousarray(tau[:, :, A][:, :, :, B]).reshape(no2, len(A) * len(B))
        prod = (np.ascontiguousarray(t.real) @ m) + 1j * (np.ascontiguousarray(t.imag) @ m)
        out[np.ix_(np.arange(tau.shape[0]), np.arange(tau.shape[1]), A, B)] = prod.reshape(
            tau.shape[0], tau.shape[1], len(A), len(B))
    return out
