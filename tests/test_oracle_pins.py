"""Pins of the CPU oracle against facts that do not come from the oracle itself.

Each test names the passage of arXiv 2301.04249 it checks.  The GPU path is
not involved; these run on the CPU only.
"""
import itertools
import os

import math

import numpy as np
import pytest

from oracle import ccsd, fockspace, memory, propagate, reference
from synthetic import Shape, draw_system

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _system(o, v, q, cfg, scale, na=None, nb=None, core=(0, 1)):
    eps, chol = draw_system(Shape(o, v, q), cfg=cfg, chol_scale=scale)
    na = o if na is None else na
    nb = o if nb is None else nb
    return reference.n_minus_one_reference(eps, chol, na, nb, core[0], core[1])


def _random_amplitudes(sys, seed, scale=0.1):
    rng = np.random.default_rng(seed)
    no, nv = sys.no, sys.nv
    t1 = (rng.standard_normal((no, nv)) + 1j * rng.standard_normal((no, nv))) * scale
    t2 = (rng.standard_normal((no, no, nv, nv)) + 1j * rng.standard_normal((no, no, nv, nv))) * scale
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    # zero the amplitudes that spin symmetry forbids (their residual is zero too)
    spin = lambda idx: idx // sys.n  # noqa: E731
    so, sv = spin(sys.occ), spin(sys.vir)
    t1 = t1 * (so[:, None] == sv[None, :])
    allowed = ((so[:, None, None, None] + so[None, :, None, None])
               == (sv[None, None, :, None] + sv[None, None, None, :]))
    same = ((so[:, None, None, None] == sv[None, None, :, None]) & (so[None, :, None, None] == sv[None, None, None, :])) | \
           ((so[:, None, None, None] == sv[None, None, None, :]) & (so[None, :, None, None] == sv[None, None, :, None]))
    t2 = t2 * (allowed & same)
    return t1, t2


# ---------------------------------------------------------------- P1 ----------
@pytest.mark.parametrize("case", [
    dict(o=3, v=3, na=3, nb=3, core=(0, 1)),   # closed-shell N, beta core hole
    dict(o=3, v=3, na=3, nb=2, core=(1, 0)),   # open-shell N, alpha hole
    dict(o=3, v=3, na=2, nb=3, core=(0, 1)),
])
def test_residual_and_energy_match_determinant_space(case):
    """Eqs. dt1eom/dt2eom and cum_gf3: projections of e^{-T} H_N e^{T} by brute force.

    Random complex T1 and T2 with a non-canonical (N-1) Fock matrix exercise
    every term of the closed-form residual; a dropped term, a wrong sign or a
    swapped index changes R by O(1) against the 1e-12 tolerance.
    """
    sys = _system(case["o"], case["v"], 10, cfg=99, scale=3.0, na=case["na"], nb=case["nb"],
                  core=case["core"])
    assert np.abs(sys.fblock("ov")).max() > 1e-3   # f_ia != 0: non-HF reference
    t1, t2 = _random_amplitudes(sys, seed=5)
    r1b, r2b, eb = fockspace.projections(sys, t1, t2)
    r1, r2 = ccsd.residual(sys, t1, t2)
    e = ccsd.energy(sys, t1, t2)
    assert np.abs(r1 - r1b).max() < 1e-12 * max(1.0, np.abs(r1b).max())
    assert np.abs(r2 - r2b).max() < 1e-12 * max(1.0, np.abs(r2b).max())
    assert abs(e - eb) < 1e-12
    assert np.abs(r2b).max() > 1.0 and np.abs(r1b).max() > 0.5


def test_residual_brute_force_unconstrained_amplitudes():
    """The projection is linear-algebra exact for any T, including spin-forbidden entries."""
    sys = _system(2, 3, 8, cfg=97, scale=3.0)
    rng = np.random.default_rng(11)
    no, nv = sys.no, sys.nv
    t1 = (rng.standard_normal((no, nv)) + 1j * rng.standard_normal((no, nv))) * 0.2
    t2 = (rng.standard_normal((no, no, nv, nv)) + 1j * rng.standard_normal((no, no, nv, nv))) * 0.2
    t2 = t2 - t2.transpose(1, 0, 2, 3)
    t2 = t2 - t2.transpose(0, 1, 3, 2)
    r1b, r2b, eb = fockspace.projections(sys, t1, t2)
    r1, r2 = ccsd.residual(sys, t1, t2)
    assert np.abs(r1 - r1b).max() < 1e-12 * np.abs(r1b).max()
    assert np.abs(r2 - r2b).max() < 1e-12 * np.abs(r2b).max()
    assert abs(ccsd.energy(sys, t1, t2) - eb) < 1e-12


# ---------------------------------------------------------------- P2 ----------
def test_cholesky_integrals_against_explicit_loops():
    """Sec. 2.3: (pq|rs) = sum_Q L^Q_pq L^Q_rs; spin-orbital <pq||rs> by explicit loops."""
    eps, chol = draw_system(Shape(2, 2, 5), cfg=3)
    n = eps.size
    eri = reference.coulomb_from_cholesky(chol)
    g = reference.antisymmetrized_spin_orbital(eri)
    for p, q, r, s in itertools.product(range(2 * n), repeat=4):
        sp, sq, sr, ss = p // n, q // n, r // n, s // n
        P, Q, R, S = p % n, q % n, r % n, s % n
        direct = sum(chol[k, P, R] * chol[k, Q, S] for k in range(chol.shape[0])) if (sp == sr and sq == ss) else 0.0
        exch = sum(chol[k, P, S] * chol[k, Q, R] for k in range(chol.shape[0])) if (sp == ss and sq == sr) else 0.0
        assert abs(g[p, q, r, s] - (direct - exch)) < 1e-14
    # eight-fold permutational symmetry of real (pq|rs)
    assert np.allclose(eri, eri.transpose(1, 0, 2, 3))
    assert np.allclose(eri, eri.transpose(2, 3, 0, 1))


def test_fock_of_n_minus_one_reference():
    """f_pq = eps_p delta_pq - <pc||qc>; for the opposite spin of c only the Coulomb part survives."""
    eps, chol = draw_system(Shape(3, 4, 9), cfg=4)
    n = eps.size
    sys = reference.n_minus_one_reference(eps, chol, 3, 3, 0, 1)
    eri = reference.coulomb_from_cholesky(chol)
    fa = sys.fock[:n, :n]
    fb = sys.fock[n:, n:]
    assert np.allclose(fa, np.diag(eps) - eri[:, :, 0, 0], atol=1e-14)
    assert np.allclose(fb, np.diag(eps) - eri[:, :, 0, 0] + eri[:, 0, 0, :], atol=1e-14)
    assert np.abs(sys.fock[:n, n:]).max() == 0.0
    assert n in sys.vir and n not in sys.occ        # beta core orbital joined the virtuals


# ---------------------------------------------------------------- P4 ----------
def test_initial_conditions_and_antisymmetry():
    """Sec. 3: T1 = T2 = 0 at tau = 0, so E = 0 and C(0) = 0; R(0) = (f_ia, <ij||ab>)."""
    sys = _system(3, 5, 12, cfg=0, scale=1.0)
    t1, t2 = ccsd.zero_amplitudes(sys)
    r1, r2 = ccsd.residual(sys, t1, t2)
    assert np.array_equal(r1, sys.fblock("ov"))
    assert np.array_equal(r2, sys.block("oovv"))
    assert ccsd.energy(sys, t1, t2) == 0
    tr = propagate.propagate(sys, 0.01, 3, tol=1e-12)
    assert tr.cumulant[0] == 0
    t2n = tr.t2
    assert np.abs(t2n + t2n.transpose(1, 0, 2, 3)).max() < 1e-15
    assert np.abs(t2n + t2n.transpose(0, 1, 3, 2)).max() < 1e-15
    ta, tb = _random_amplitudes(sys, 3)
    _, r2 = ccsd.residual(sys, ta, tb)
    assert np.abs(r2 + r2.transpose(1, 0, 2, 3)).max() < 1e-13
    assert np.abs(r2 + r2.transpose(0, 1, 3, 2)).max() < 1e-13


# ---------------------------------------------------------------- P5 ----------
def test_short_time_closed_form():
    """C(tau) = -(tau^2/2) <Phi|H_N^2|Phi> + O(tau^3) (Eq. cum_gf3 with T ~ i tau R(0)).

    <Phi|H_N^2|Phi> = sum |f_ia|^2 + 1/4 sum <ij||ab>^2, independent of the oracle's residual.
    """
    sys = _system(3, 6, 12, cfg=0, scale=1.0)
    s = np.sum(sys.fblock("ov") ** 2) + 0.25 * np.sum(sys.block("oovv") ** 2)
    ratios = []
    for dt in (1e-3, 5e-4, 2.5e-4):
        tr = propagate.propagate(sys, dt, 1, tol=1e-14, max_iter=100)
        ratios.append(tr.cumulant[1] / (-0.5 * dt * dt * s))
    dev = [abs(r - 1) for r in ratios]
    assert dev[-1] < 1e-2
    assert dev[0] / dev[1] > 1.8 and dev[1] / dev[2] > 1.8   # O(dt) relative correction


def test_short_time_hn_squared_brute_force():
    """The S of the closed form equals <Phi|H_N^2|Phi> from the determinant-space Hamiltonian."""
    sys = _system(2, 3, 8, cfg=1, scale=2.0)
    sector = fockspace.Sector(sys.nso, sys.no)
    H = fockspace.hamiltonian(sys, sector)
    k = sector.index[fockspace.reference_det(sys)]
    HN = H - H[k, k] * np.eye(sector.dim)
    s_brute = (HN @ HN)[k, k]
    s = np.sum(sys.fblock("ov") ** 2) + 0.25 * np.sum(sys.block("oovv") ** 2)
    assert abs(s - s_brute) < 1e-12 * s_brute


# ---------------------------------------------------------------- P6 ----------
@pytest.mark.parametrize("occ", [(2, 1, 0, 0), (3, 0, 1, 0)])
def test_two_electron_exactness(occ):
    """With two electrons CCSD is full CI: e^{C(tau)} = <Phi|e^{i H_N tau}|Phi> up to O(dt^2).

    Exact diagonalisation of H in the two-electron sector supplies the reference
    (Eqs. N_c, cum_gf3: N_c = e^{i E_ref tau} e^{C}).
    """
    na, nb, co, cs = occ
    eps, chol = draw_system(Shape(2, 4, 12), cfg=98, chol_scale=3.0)
    sys = reference.n_minus_one_reference(eps, chol, na, nb, co, cs)
    assert sys.no == 2
    tau = 0.5
    errs = []
    cs_ = []
    for dt in (0.01, 0.005, 0.0025):
        n = int(round(tau / dt))
        tr = propagate.propagate(sys, dt, n, tol=1e-12, max_iter=200)
        ex = fockspace.exact_overlap(sys, tr.times)
        errs.append(abs(np.exp(tr.cumulant[-1]) - ex[-1]))
        cs_.append(np.exp(tr.cumulant[-1]))
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5
    richardson = (4 * cs_[2] - cs_[1]) / 3
    assert abs(richardson - ex[-1]) < 0.05 * errs[2]


# ---------------------------------------------------------------- P7 ----------
def test_spin_flip_invariance():
    """A closed-shell N reference: a core hole in alpha or in beta gives the same C(t)."""
    eps, chol = draw_system(Shape(3, 5, 12), cfg=0)
    a = reference.n_minus_one_reference(eps, chol, 3, 3, 0, 0)
    b = reference.n_minus_one_reference(eps, chol, 3, 3, 0, 1)
    ta = propagate.propagate(a, 0.025, 8, fixed_iters=4)
    tb = propagate.propagate(b, 0.025, 8, fixed_iters=4)
    assert np.abs(ta.cumulant - tb.cumulant).max() < 1e-13
    assert np.abs(ta.cumulant).max() > 1e-3


# ---------------------------------------------------------------- P8 ----------
def test_integrator_order():
    """Eq. trapzrule: observed convergence order of C(tau) is >= 0.9 (the trapezoid gives ~2)."""
    sys = _system(2, 4, 10, cfg=0, scale=1.0)
    tau = 0.32
    ref = propagate.propagate(sys, 0.04 / 64, 64 * 8, tol=1e-13, max_iter=100).cumulant[-1]
    errs = []
    for k in (1, 2, 4):
        dt = 0.04 / k
        c = propagate.propagate(sys, dt, 8 * k, tol=1e-13, max_iter=100).cumulant[-1]
        errs.append(abs(c - ref))
    p1 = np.log2(errs[0] / errs[1])
    p2 = np.log2(errs[1] / errs[2])
    assert p1 > 0.9 and p2 > 0.9
    assert 1.7 < p2 < 2.3
    del tau


# ---------------------------------------------------------------- P9 ----------
def test_fixed_point_maps_agree():
    """The plain and the denominator map share the fixed point of Eq. trapzrule."""
    sys = _system(3, 5, 12, cfg=0, scale=1.0)
    t1, t2 = _random_amplitudes(sys, 7, scale=0.01)
    a1, a2, _ = propagate.trapezoid_step(sys, t1, t2, 0.02, tol=1e-14, max_iter=200, fp_map="plain")
    b1, b2, _ = propagate.trapezoid_step(sys, t1, t2, 0.02, tol=1e-14, max_iter=200, fp_map="denominator")
    assert np.abs(a1 - b1).max() < 1e-12
    assert np.abs(a2 - b2).max() < 1e-12
    # and both satisfy the implicit equation itself
    h = 0.01j
    r0 = ccsd.residual(sys, t1, t2)
    r1 = ccsd.residual(sys, a1, a2)
    assert np.abs(a2 - (t2 + h * (r0[1] + r1[1]))).max() < 1e-12


# ---------------------------------------------------------------- P10 ---------
def test_table2_t2_memory():
    """Table 2, T2 column: full aa+bb+ab complex128 blocks in GiB per timeline tensor."""
    rows = []
    with open(os.path.join(GOLDEN, "table2_t2_memory.txt")) as fh:
        for line in fh:
            if line.startswith("#") or not line.strip():
                continue
            name, oa, ob, va, vb, gb = line.split()
            rows.append((name, int(oa), int(ob), int(va), int(vb), float(gb)))
    assert len(rows) == 4
    for name, oa, ob, va, vb, gb in rows:
        assert abs(memory.t2_gib(oa, ob, va, vb) - gb) < 0.1, name


# ---------------------------------------------------------------- P11 ---------
def test_noninteracting_limit():
    """L = 0: f = diag(eps), R(T) = -D*T, so T stays 0 and C stays 0 (Fock definition, Sec. 2.1)."""
    eps, chol = draw_system(Shape(3, 4, 6), cfg=0)
    sys = reference.n_minus_one_reference(eps, 0 * chol, 3, 3, 0, 1)
    assert np.array_equal(sys.fock, np.diag(np.concatenate([eps, eps])))
    tr = propagate.propagate(sys, 0.05, 5, fixed_iters=3)
    assert np.abs(tr.cumulant).max() == 0.0
    t1, t2 = _random_amplitudes(sys, 1)
    r1, r2 = ccsd.residual(sys, t1, t2)
    d1, d2 = propagate._denominators(sys)
    assert np.abs(r1 + d1 * t1).max() < 1e-14
    assert np.abs(r2 + d2 * t2).max() < 1e-14


def test_energy_fT1_reading():
    """Eq. cum_gf3 vs the printed Eq. dcdt: they differ by exactly sum_ia f_ia t_ia."""
    sys = _system(3, 5, 12, cfg=0, scale=1.0)
    t1, t2 = _random_amplitudes(sys, 9)
    d = ccsd.energy(sys, t1, t2, True) - ccsd.energy(sys, t1, t2, False)
    assert abs(d - np.sum(sys.fblock("ov") * t1)) < 1e-14


def test_green_function_and_spectrum_free_particle():
    """C = 0: G = -i e^{-i eps_c tau}; A(omega) is a Lorentzian of width eta at eps_c (Eq. cum_gf)."""
    times = np.arange(0, 4000) * 0.05
    g = propagate.green_function(times, np.zeros_like(times, dtype=complex), -20.0)
    omegas = np.linspace(-20.5, -19.5, 1001)
    eta = 0.05
    a = propagate.spectral_function(times, g, omegas, eta)
    peak = propagate.qp_peak(omegas, a)
    assert abs(peak - (-20.0)) < 1e-4
    lorentz = eta / np.pi / ((omegas + 20.0) ** 2 + eta ** 2)
    assert np.abs(a - lorentz).max() < 2e-2 * lorentz.max()


def test_spectrum_of_linear_cumulant_closed_form():
    """Eqs. cum_gf, cum_gf2 with a nonzero cumulant C(tau) = (-a + i b) tau and a nonzero
    E_N^corr: every damped trapezoid term is a power z^n of one complex number, so the
    discrete transform is a geometric sum, and A = -(1/pi) Im of it in closed form.  The
    peak sits at eps_c + E_N^corr - b with half-width a + eta: the sign of C in exp(C), the
    sign of the E_N^corr phase and the trapezoid end weights all change A here."""
    dt, n = 0.05, 2400
    times = np.arange(n + 1) * dt
    a_c, b_c, eps_c, e_corr, eta = 0.04, 0.3, -20.0, -0.11, 0.02
    cum = (-a_c + 1j * b_c) * times
    g = propagate.green_function(times, cum, eps_c, e_corr)
    omegas = np.linspace(-21.0, -19.0, 801)
    a = propagate.spectral_function(times, g, omegas, eta)
    z = np.exp((1j * (omegas - eps_c - e_corr + b_c) - (a_c + eta)) * dt)
    geo = (1 - z ** (n + 1)) / (1 - z) - 0.5 * (1 + z ** n)
    closed = -(-1j * dt * geo).imag / np.pi
    assert np.abs(a - closed).max() < 1e-11 * closed.max()
    # continuum limit: a Lorentzian of half-width a + eta at eps_c + E_N^corr - b
    w0, gam = eps_c + e_corr - b_c, a_c + eta
    lorentz = gam / np.pi / ((omegas - w0) ** 2 + gam ** 2)
    assert np.abs(a - lorentz).max() < 2e-3 * lorentz.max()
    assert abs(propagate.qp_peak(omegas, a) - w0) < 2e-4


def test_qp_peak_refinement_between_grid_points():
    """The QP position is refined by the parabola through the grid maximum and its two
    neighbours: exact for samples of a parabola whose vertex lies between grid points, and
    for a Lorentzian far closer to its centre than the grid spacing."""
    omegas = np.linspace(-20.5, -19.5, 1001)        # spacing 1e-3
    h = omegas[1] - omegas[0]
    for w0 in (-20.0 + 0.37 * h, -19.9 - 0.21 * h, -20.3 + 0.49 * h):
        y = 5.0 - 3.0 * (omegas - w0) ** 2
        assert abs(propagate.qp_peak(omegas, y) - w0) < 1e-9 * h
        k = int(np.argmax(y))
        assert abs(omegas[k] - w0) > 0.2 * h           # the refinement moved the estimate
    gam, w0 = 0.01, -20.0 + 0.43 * h
    lor = gam / ((omegas - w0) ** 2 + gam ** 2)
    assert abs(propagate.qp_peak(omegas, lor) - w0) < 5e-3 * h     # raw arg-max: 0.43 h off
    # a peak on the first or last grid point is returned as it is
    assert propagate.qp_peak(omegas, -(omegas + 20.5) ** 2) == omegas[0]


def test_lean_mode_matches_dense():
    """Lean blocks and the per-spin Coulomb particle ladder equal the dense <pq||rs> path."""
    eps, chol = draw_system(Shape(3, 6, 14), cfg=5, chol_scale=2.0)
    dense = reference.n_minus_one_reference(eps, chol, 3, 3, 0, 1)
    lean = reference.n_minus_one_reference(eps, chol, 3, 3, 0, 1, lean=True)
    assert lean.g is None
    assert np.abs(dense.fock - lean.fock).max() < 1e-14
    t1, t2 = _random_amplitudes(dense, 4)
    a1, a2 = ccsd.residual(dense, t1, t2)
    b1, b2 = ccsd.residual(lean, t1, t2)
    assert np.abs(a1 - b1).max() < 1e-13 and np.abs(a2 - b2).max() < 1e-13
    assert abs(ccsd.energy(dense, t1, t2) - ccsd.energy(lean, t1, t2)) < 1e-14


def test_size_extensivity_of_residual_and_energy():
    """CCSD is size-extensive: for two parts with no integral between them (block-diagonal
    Cholesky vectors on disjoint Q ranges) and amplitudes inside each part, the residual on
    each part is that part's own residual, every element joining them vanishes, and the
    energy is the sum.  Pins the connectedness of every term of the oracle's equations."""
    o, v, q, qa = 5, 9, 24, 10
    n = o + v
    eps, chol = draw_system(Shape(o, v, q), cfg=41, chol_scale=2.0)
    in_a = np.zeros(n, dtype=bool)
    in_a[:2] = True                 # part A: occupied 0, 1 (core orbital 0) and 3 virtuals
    in_a[o:o + 3] = True
    chol[:qa] *= in_a[:, None] & in_a[None, :]
    chol[qa:] *= ~in_a[:, None] & ~in_a[None, :]
    big = reference.n_minus_one_reference(eps, chol, o, o, 0, 1)

    def part(mask, qs, hole):
        sel = np.flatnonzero(mask)
        e, c = eps[sel], np.ascontiguousarray(chol[qs][:, sel][:, :, sel])
        m, no_p = len(sel), int(np.sum(sel < o))
        if hole:
            sub = reference.n_minus_one_reference(e, c, no_p, no_p, 0, 1)
        else:                       # closed-shell N-electron part: Fock diagonal eps
            occ = np.array([p + m * s for s in (0, 1) for p in range(no_p)])
            vir = np.array(sorted(set(range(2 * m)) - set(occ.tolist())))
            sub = reference.SpinOrbitalSystem(
                n=m, eps=e, chol=c, occ=occ, vir=vir, core=-1, fock=np.diag(np.concatenate([e, e])),
                g=reference.antisymmetrized_spin_orbital(reference.coulomb_from_cholesky(c)))
        # spin-orbital of the big system -> spin-orbital of the part
        so = {int(p) + s * n: int(k) + s * m for s in (0, 1) for k, p in enumerate(sel)}
        oc = [k for k, x in enumerate(big.occ) if int(x) in so]
        vi = [k for k, x in enumerate(big.vir) if int(x) in so]
        pos_o = {int(x): k for k, x in enumerate(sub.occ)}
        pos_v = {int(x): k for k, x in enumerate(sub.vir)}
        return (sub, np.array(oc), np.array(vi), np.array([pos_o[so[int(big.occ[k])]] for k in oc]),
                np.array([pos_v[so[int(big.vir[k])]] for k in vi]))

    parts = [part(in_a, slice(None, qa), True), part(~in_a, slice(qa, None), False)]
    t1 = np.zeros((big.no, big.nv), dtype=complex)
    t2 = np.zeros((big.no, big.no, big.nv, big.nv), dtype=complex)
    amps = []
    for k, (sub, oc, vi, so_, sv_) in enumerate(parts):
        st1, st2 = _random_amplitudes(sub, 100 + k)
        assert len(so_) == sub.no and len(sv_) == sub.nv
        t1[np.ix_(oc, vi)] = st1[np.ix_(so_, sv_)]
        t2[np.ix_(oc, oc, vi, vi)] = st2[np.ix_(so_, so_, sv_, sv_)]
        amps.append((st1, st2))
    r1, r2 = ccsd.residual(big, t1, t2)
    covered1 = np.zeros(r1.shape, dtype=bool)
    covered2 = np.zeros(r2.shape, dtype=bool)
    e_sum = 0.0
    for (sub, oc, vi, so_, sv_), (st1, st2) in zip(parts, amps):
        s1, s2 = ccsd.residual(sub, st1, st2)
        assert np.abs(r1[np.ix_(oc, vi)] - s1[np.ix_(so_, sv_)]).max() < 1e-12
        assert np.abs(r2[np.ix_(oc, oc, vi, vi)] - s2[np.ix_(so_, so_, sv_, sv_)]).max() < 1e-12
        covered1[np.ix_(oc, vi)] = True
        covered2[np.ix_(oc, oc, vi, vi)] = True
        e_sum += ccsd.energy(sub, st1, st2)
    assert np.abs(r1[~covered1]).max() < 1e-13
    assert np.abs(r2[~covered2]).max() < 1e-13
    assert abs(ccsd.energy(big, t1, t2) - e_sum) < 1e-12


def test_ground_state_ccsd_exact_for_two_electrons():
    """Ground-state CCSD (E_N^corr for G(tau)) is full CI for two electrons: the correlation
    energy equals the lowest eigenvalue of H in the two-electron sector minus <Phi|H|Phi>."""
    from oracle import groundstate
    eps, chol = draw_system(Shape(1, 5, 14), cfg=77, chol_scale=2.0)
    sysm = reference.closed_shell_reference(eps, chol, 1, 1)
    e_cc, t1, t2, it = groundstate.solve(sysm, tol=1e-13, max_iter=500)
    sector = fockspace.Sector(sysm.nso, 2)
    H = fockspace.hamiltonian(sysm, sector)
    ref = sector.index[fockspace.reference_det(sysm)]
    e_fci = np.linalg.eigvalsh(H)[0] - H[ref, ref]
    assert abs(e_cc.imag) < 1e-14
    assert e_fci < -1e-3                         # a correlated case
    assert abs(e_cc.real - e_fci) < 1e-10 * abs(e_fci)
    assert np.abs(t1.imag).max() == 0 and np.abs(t2.imag).max() == 0


def test_ground_state_ccsd_weak_coupling_is_mp2():
    """As the integrals are scaled down by lam, E_CCSD / E_MP2 - 1 = O(lam^2) (MP3 and
    higher orders): the deviation drops ~4x per halving of lam."""
    from oracle import groundstate
    devs = []
    for lam in (0.2, 0.1, 0.05):
        eps, chol = draw_system(Shape(3, 5, 12), cfg=78, chol_scale=lam)
        sysm = reference.closed_shell_reference(eps, chol, 3, 3)
        e_cc = groundstate.solve(sysm, tol=1e-15, max_iter=500)[0].real
        devs.append(abs(e_cc / groundstate.mp2_energy(sysm) - 1.0))
    assert devs[0] / devs[1] > 3.0 and devs[1] / devs[2] > 3.0
    assert devs[2] < 1e-3


def test_satellites_of_a_single_mode_cumulant():
    """A cumulant with one bosonic mode, C(tau) = (-a + i b) tau + lam (e^{i W tau} - 1), makes
    G(tau) a Poisson series of damped exponentials (Eqs. cum_gf, cum_gf2): A(omega) is a
    QP Lorentzian at eps_c + E_N^corr - b and satellites n = 1, 2, ... at n W below it, with
    weights lam^n / n! relative to the QP line.  The peak extraction finds them in that order
    at those positions and height ratios (the sign of W in C decides on which side the
    satellites lie; dropping the 1/n! or the Poisson factor changes the ratios)."""
    dt, n = 0.05, 6000
    times = np.arange(n + 1) * dt
    a_c, b_c, lam, om, eps_c, e_corr, eta = 0.015, 0.3, 0.6, 0.8, -20.0, -0.11, 0.01
    cum = (-a_c + 1j * b_c) * times + lam * (np.exp(1j * om * times) - 1.0)
    g = propagate.green_function(times, cum, eps_c, e_corr)
    omegas = np.arange(-23.5, -19.0, 0.002)
    a = propagate.spectral_function(times, g, omegas, eta)
    peaks = propagate.spectral_peaks(omegas, a, 4)
    w0 = eps_c + e_corr - b_c
    expect = [w0 - k * om for k in range(4)]
    assert np.abs(peaks[:, 0] - expect).max() < 2e-4
    ratios = peaks[1:, 1] / peaks[0, 1]
    poisson = np.array([lam ** k / math.factorial(k) for k in range(1, 4)])
    assert np.abs(ratios / poisson - 1).max() < 2e-2
    # the same extraction takes the global maximum first, as qp_peak does
    assert abs(peaks[0, 0] - propagate.qp_peak(omegas, a)) < 1e-12
