"""CCSD amplitude residual and cumulant derivative in spin-orbital form.

Paper, Eqs. dt1eom / dt2eom: -i d/dt t_x = <Phi_x| (H_N e^{T1+T2})_C |Phi>,
x = singles, doubles.  The paper gives only this definition; the closed form
below is the textbook spin-orbital CCSD projection for a general
(non-canonical) Fock operator, in the intermediate form of Stanton, Gauss,
Watts and Bartlett (J. Chem. Phys. 94, 4334 (1991)).  It is pinned against a
brute-force determinant-space evaluation of the definition
(tests/test_oracle_pins.py).

The residual returned is R = RHS - D*t (D_ia = f_ii - f_aa,
D_ijab = f_ii + f_jj - f_aa - f_bb), i.e. exactly <Phi_x|e^{-T} H_N e^{T}|Phi>.
Integrals are real; amplitudes are complex; no complex conjugation appears.

Cumulant derivative (Eq. cum_gf3): -i dC/dt = <Phi|(H_N e^T)_C|Phi>
  = sum f_ia t_ia + 1/4 sum <ij||ab> t_ijab + 1/2 sum <ij||ab> t_ia t_jb.
Eq. dcdt prints only the T2 and T1*T1 parts; ``include_fT1=False`` gives that
literal reading (the two agree whenever f_ia = 0).
"""
from __future__ import annotations

import numpy as np

from .reference import SpinOrbitalSystem, particle_ladder


def _blocks(sys: SpinOrbitalSystem):
    b = {}
    for spec in ("oooo", "ooov", "oovv", "ovov", "ovvo", "ovvv", "vovv", "oovo",
                 "vvvo", "ovoo"):
        b[spec] = sys.block(spec)
    for spec in ("oo", "ov", "vv"):
        b["f" + spec] = sys.fblock(spec)
    return b


def _perm_ij(x):
    """P(ij) X_ij.. = X_ij.. - X_ji.. on a [i,j,a,b] array."""
    return x - x.transpose(1, 0, 2, 3)


def _perm_ab(x):
    return x - x.transpose(0, 1, 3, 2)


def residual(sys: SpinOrbitalSystem, t1: np.ndarray, t2: np.ndarray, blocks=None):
    """Return (R1[i,a], R2[i,j,a,b]) = <Phi_x| e^{-T} H_N e^{T} |Phi>."""
    b = blocks if blocks is not None else _blocks(sys)
    foo, fov, fvv = b["foo"], b["fov"], b["fvv"]
    oooo, ooov, oovv = b["oooo"], b["ooov"], b["oovv"]
    ovvo, ovvv = b["ovvo"], b["ovvv"]
    vovv, oovo, vvvo, ovoo = b["vovv"], b["oovo"], b["vvvo"], b["ovoo"]
    ein = lambda s, *a: np.einsum(s, *a, optimize=True)  # noqa: E731

    no = foo.shape[0]
    nv = fvv.shape[0]
    # tau-tilde and tau (Stanton-Gauss Eqs. 9-10)
    t1t1 = ein("ia,jb->ijab", t1, t1)
    tau_t = t2 + 0.5 * (t1t1 - t1t1.transpose(0, 1, 3, 2))
    tau = t2 + t1t1 - t1t1.transpose(0, 1, 3, 2)

    # One-body intermediates.  The diagonal Fock elements are kept in F_ae and
    # F_mi here and removed again below, so that R = RHS - D*t holds exactly.
    eye_o = np.eye(no)
    eye_v = np.eye(nv)
    fae = (fvv * (1 - eye_v)
           - 0.5 * ein("me,ma->ae", fov, t1)
           + ein("mf,mafe->ae", t1, b["ovvv"])
           - 0.5 * ein("mnaf,mnef->ae", tau_t, oovv))
    fmi = (foo * (1 - eye_o)
           + 0.5 * ein("ie,me->mi", t1, fov)
           + ein("ne,mnie->mi", t1, ooov)
           + 0.5 * ein("inef,mnef->mi", tau_t, oovv))
    fme = fov + ein("nf,mnef->me", t1, oovv)

    # Two-body intermediates
    wmnij = (oooo
             + _perm_ij_last(ein("je,mnie->mnij", t1, ooov))
             + 0.25 * ein("ijef,mnef->mnij", tau, oovv))
    # W_abef = <ab||ef> - P(ab) t_m^b <am||ef> + 1/4 tau_mn^ab <mn||ef> enters only
    # through 1/2 sum_ef tau_ij^ef W_abef, evaluated below term by term so that
    # no (virtual)^4 intermediate is formed.
    wmbej = (ovvo
             + ein("jf,mbef->mbej", t1, ovvv)
             - ein("nb,mnej->mbej", t1, oovo)
             - ein("jnfb,mnef->mbej", 0.5 * t2 + ein("jf,nb->jnfb", t1, t1), oovv))

    # T1 residual (Stanton-Gauss Eq. 1)
    r1 = (fov.copy()
          + ein("ie,ae->ia", t1, fae)
          - ein("ma,mi->ia", t1, fmi)
          + ein("imae,me->ia", t2, fme)
          - ein("nf,naif->ia", t1, b["ovov"])
          - 0.5 * ein("imef,maef->ia", t2, ovvv)
          - 0.5 * ein("mnae,nmei->ia", t2, oovo))
    dia = np.diag(foo)[:, None] - np.diag(fvv)[None, :]
    r1 = r1 - dia * t1

    # T2 residual (Stanton-Gauss Eq. 2)
    fbe_eff = fae - 0.5 * ein("mb,me->be", t1, fme)
    fmj_eff = fmi + 0.5 * ein("je,me->mj", t1, fme)
    r2 = oovv.astype(complex).copy()
    r2 = r2 + _perm_ab(ein("ijae,be->ijab", t2, fbe_eff))
    r2 = r2 - _perm_ij(ein("imab,mj->ijab", t2, fmj_eff))
    r2 = r2 + 0.5 * ein("mnab,mnij->ijab", tau, wmnij)
    r2 = r2 + particle_ladder(sys, tau)
    r2 = r2 - _perm_ab(ein("mb,ijam->ijab", t1, 0.5 * ein("ijef,amef->ijam", tau, vovv)))
    r2 = r2 + 0.125 * ein("mnab,ijmn->ijab", tau, ein("ijef,mnef->ijmn", tau, oovv))
    ring = ein("imae,mbej->ijab", t2, wmbej) - ein("ie,ma,mbej->ijab", t1, t1, ovvo)
    r2 = r2 + _perm_ij(_perm_ab(ring))
    r2 = r2 + _perm_ij(ein("ie,abej->ijab", t1, vvvo))
    r2 = r2 - _perm_ab(ein("ma,mbij->ijab", t1, ovoo))
    fo = np.diag(foo)
    fv = np.diag(fvv)
    dijab = fo[:, None, None, None] + fo[None, :, None, None] - fv[None, None, :, None] - fv[None, None, None, :]
    r2 = r2 - dijab * t2
    return r1, r2


def _perm_ij_last(x):
    """P(ij) on a [m,n,i,j] array."""
    return x - x.transpose(0, 1, 3, 2)


def _perm_ab_first(x):
    """P(ab) on an [a,b,e,f] array."""
    return x - x.transpose(1, 0, 2, 3)


def energy(sys: SpinOrbitalSystem, t1: np.ndarray, t2: np.ndarray, include_fT1: bool = True):
    """<Phi|(H_N e^T)_C|Phi> (Eq. cum_gf3); ``include_fT1=False`` drops sum f_ia t_ia (Eq. dcdt)."""
    fov = sys.fblock("ov")
    oovv = sys.block("oovv")
    e = 0.25 * np.einsum("ijab,ijab->", oovv, t2) + 0.5 * np.einsum("ijab,ia,jb->", oovv, t1, t1)
    if include_fT1:
        e = e + np.einsum("ia,ia->", fov, t1)
    return complex(e)


def zero_amplitudes(sys: SpinOrbitalSystem):
    return (np.zeros((sys.no, sys.nv), dtype=complex),
            np.zeros((sys.no, sys.no, sys.nv, sys.nv), dtype=complex))
