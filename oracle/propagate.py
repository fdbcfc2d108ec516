"""Time propagation of the CCSD amplitudes and the cumulant.

Paper, Sec. 3 (Eq. trapzrule): the amplitudes obey -i dt/dtau = R(T)
(Eqs. dt1eom/dt2eom), i.e. dT/dtau = i R(T), integrated with the implicit
trapezoidal rule ("first-order Adams-Moulton")

    T_{n+1} = T_n + (i dt / 2) [R(T_n) + R(T_{n+1})],   T(0) = 0,

solved by fixed-point iteration.  The cumulant follows Eq. cum_gf3,
dC/dtau = i E(T), accumulated with the same trapezoidal weights on the same
grid, C(0) = 0.  G(tau) and A(omega) follow Eqs. cum_gf / cum_gf2 and
A = -(1/pi) Im G(omega).

Readings where the paper is silent (stated once here, used everywhere):
* fixed point: T^(0) = T_n, T^(k+1) = T_n + (i dt/2)(R(T_n) + R(T^(k)));
  either exactly ``fixed_iters`` passes, or until max|T^(k+1) - T^(k)| < tol
  over all amplitudes (failure after ``max_iter`` passes raises);
  T_{n+1} is the last iterate.
* "denominator" map: with R = R' - D*T the same fixed point is reached by
  T^(k+1) = [T_n + (i dt/2)(R(T_n) + R'(T^(k)))] / (1 + (i dt/2) D).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from . import ccsd
from .reference import SpinOrbitalSystem


class NoConvergence(RuntimeError):
    pass


@dataclasses.dataclass
class Trajectory:
    times: np.ndarray          # [n_steps+1]
    cumulant: np.ndarray       # [n_steps+1] complex
    energies: np.ndarray       # [n_steps+1] complex E(T_n)
    iters: np.ndarray          # [n_steps] micro-iterations per step
    t1: np.ndarray
    t2: np.ndarray


def _denominators(sys: SpinOrbitalSystem):
    fo = np.diag(sys.fblock("oo"))
    fv = np.diag(sys.fblock("vv"))
    d1 = fo[:, None] - fv[None, :]
    d2 = fo[:, None, None, None] + fo[None, :, None, None] - fv[None, None, :, None] - fv[None, None, None, :]
    return d1, d2


def trapezoid_step(sys, t1, t2, dt, r_n=None, fixed_iters=None, tol=1e-13, max_iter=50,
                   fp_map="plain", blocks=None):
    """One implicit trapezoidal step from T_n = (t1, t2).  Returns (t1', t2', n_iter)."""
    if r_n is None:
        r_n = ccsd.residual(sys, t1, t2, blocks)
    h = 0.5j * dt
    rhs1 = t1 + h * r_n[0]
    rhs2 = t2 + h * r_n[1]
    if fp_map == "denominator":
        d1, d2 = _denominators(sys)
        den1 = 1.0 + h * d1
        den2 = 1.0 + h * d2
    cur1, cur2, r_cur = t1, t2, r_n
    n_pass = fixed_iters if fixed_iters is not None else max_iter
    for k in range(n_pass):
        if k > 0:
            r_cur = ccsd.residual(sys, cur1, cur2, blocks)
        if fp_map == "plain":
            nxt1 = rhs1 + h * r_cur[0]
            nxt2 = rhs2 + h * r_cur[1]
        elif fp_map == "denominator":
            # R'(T) = R(T) + D*T
            nxt1 = (rhs1 + h * (r_cur[0] + d1 * cur1)) / den1
            nxt2 = (rhs2 + h * (r_cur[1] + d2 * cur2)) / den2
        else:
            raise ValueError(fp_map)
        delta = max(np.max(np.abs(nxt1 - cur1), initial=0.0), np.max(np.abs(nxt2 - cur2), initial=0.0))
        cur1, cur2 = nxt1, nxt2
        if fixed_iters is None and delta < tol:
            return cur1, cur2, k + 1
    if fixed_iters is None:
        raise NoConvergence(f"fixed point not converged after {max_iter} passes (last change {delta:.3e})")
    return cur1, cur2, n_pass


def propagate(sys: SpinOrbitalSystem, dt: float, n_steps: int, fixed_iters=None, tol=1e-13,
              max_iter=50, fp_map="plain", include_fT1=True, t1=None, t2=None) -> Trajectory:
    """Propagate from T(0) (zero unless given) for n_steps; C by the trapezoidal rule."""
    blocks = ccsd._blocks(sys)
    if t1 is None:
        t1, t2 = ccsd.zero_amplitudes(sys)
    times = dt * np.arange(n_steps + 1)
    cum = np.zeros(n_steps + 1, dtype=complex)
    ens = np.zeros(n_steps + 1, dtype=complex)
    iters = np.zeros(n_steps, dtype=np.int64)
    ens[0] = ccsd.energy(sys, t1, t2, include_fT1)
    for n in range(n_steps):
        t1, t2, k = trapezoid_step(sys, t1, t2, dt, fixed_iters=fixed_iters, tol=tol,
                                   max_iter=max_iter, fp_map=fp_map, blocks=blocks)
        iters[n] = k
        ens[n + 1] = ccsd.energy(sys, t1, t2, include_fT1)
        cum[n + 1] = cum[n] + 0.5j * dt * (ens[n] + ens[n + 1])
    return Trajectory(times=times, cumulant=cum, energies=ens, iters=iters, t1=t1, t2=t2)


def green_function(times, cumulant, eps_core: float, e_corr_n: float = 0.0):
    """G(tau) = -i exp(-i (eps_c + E_N^corr) tau) exp(C(tau)) for tau >= 0 (Eqs. cum_gf, cum_gf2)."""
    times = np.asarray(times)
    return -1j * np.exp(-1j * (eps_core + e_corr_n) * times) * np.exp(np.asarray(cumulant))


def spectral_function(times, g, omegas, eta: float):
    """A(omega) = -(1/pi) Im G(omega), G(omega) = int_0^T dtau e^{i omega tau} e^{-eta tau} G(tau).

    The integral uses trapezoidal weights on the propagation grid; eta is a
    damping (Lorentzian broadening) chosen by the caller.
    """
    times = np.asarray(times)
    g = np.asarray(g)
    w = np.full(times.shape, times[1] - times[0]) if times.size > 1 else np.zeros(1)
    w[0] *= 0.5
    w[-1] *= 0.5
    phase = np.exp(1j * np.outer(np.asarray(omegas), times) - eta * times[None, :])
    gw = phase @ (w * g)
    return -gw.imag / np.pi


def qp_peak(omegas, spectrum):
    """Position of the largest peak, refined by a parabola through the three top samples."""
    omegas = np.asarray(omegas)
    a = np.asarray(spectrum)
    k = int(np.argmax(a))
    if 0 < k < a.size - 1:
        y0, y1, y2 = a[k - 1], a[k], a[k + 1]
        den = y0 - 2 * y1 + y2
        shift = 0.5 * (y0 - y2) / den if den != 0 else 0.0
        return float(omegas[k] + shift * (omegas[1] - omegas[0]))
    return float(omegas[k])


def spectral_peaks(omegas, spectrum, k):
    """The quasi-particle peak and its satellites: the local maxima of A on a uniform grid
    (A_j > A_{j-1} and A_j >= A_{j+1} at interior points), the largest first (the first index
    on ties), at most k, each refined like qp_peak by the parabola through the maximum and
    its two neighbours.  Returns an array [n][2] of (position, A at the grid maximum)."""
    omegas = np.asarray(omegas)
    a = np.asarray(spectrum)
    j = np.arange(1, a.size - 1)
    local = j[(a[1:-1] > a[:-2]) & (a[1:-1] >= a[2:])]
    chosen = sorted(local.tolist(), key=lambda x: (-a[x], x))[:k]
    out = []
    for x in chosen:
        y0, y1, y2 = a[x - 1], a[x], a[x + 1]
        den = y0 - 2 * y1 + y2
        shift = 0.5 * (y0 - y2) / den if den != 0 else 0.0
        out.append((float(omegas[x] + shift * (omegas[1] - omegas[0])), float(a[x])))
    return np.array(out, dtype=float).reshape(-1, 2)
