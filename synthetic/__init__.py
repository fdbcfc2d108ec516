"""Seeded synthetic inputs for the RT-EOM-CCSD hot path.

This module is the single source of inputs for both the GPU path and the CPU
oracle.  It holds random draws only, none of the method's arithmetic: orbital
energies, Cholesky vectors and (optionally) amplitudes of a stated shape and
distribution.  The molecules of the paper (formaldehyde, ESCA, Zn-porphyrin;
Sec. "Geometries, Basis Sets, and Computational Details" and Table 2) are not
available, so these draws stand in for their integrals.

Recipe (every array is float64):

* ``eps`` [n]: the N-electron orbital energies (Fock diagonal).  Index 0 is the
  core orbital at -20 Eh; occupied 1..o-1 are U[-2, -0.3] sorted ascending;
  virtuals o..n-1 are U[0.1, 3] sorted ascending.
* ``chol`` [Q][n][n]: Cholesky vectors, symmetric in (p, q).  For vector q
  (0-based) the upper triangle p <= r is drawn q-major from N(0, 1) and scaled
  by ``0.1 * exp(-q / 16) * chol_scale``, then mirrored.
* amplitudes (only when asked): real and imaginary parts independently
  N(0, sigma^2).

The generator is ``numpy.random.default_rng(SeedSequence([2301, 4249, cfg,
sys]))`` with the draw order above, so every consumer sees the same numbers.
"""
from __future__ import annotations

import dataclasses

import numpy as np

CORE_EPS = -20.0


@dataclasses.dataclass(frozen=True)
class Shape:
    """N-electron closed-shell shape: o occupied and v virtual orbitals per spin."""

    o: int
    v: int
    nchol: int

    @property
    def n(self) -> int:
        return self.o + self.v


# Workload shapes (per spin, N-electron).  The names say what each one mirrors.
TINY = Shape(o=4, v=16, nchol=48)
FORMALDEHYDE = Shape(o=8, v=110, nchol=600)
ESCA = Shape(o=71, v=649, nchol=2000)
# The paper's ESCA spectra run has 71 occupied and 649 virtual spin-orbitals in
# total (abstract): 36 + 35 occupied, 324 + 325 virtual with the beta hole.
ESCA_PAPER = Shape(o=36, v=324, nchol=2000)
ZN_PORPHYRIN = Shape(o=95, v=560, nchol=3000)


def rng_for(cfg: int, sys_id: int = 0) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([2301, 4249, int(cfg), int(sys_id)]))


def draw_system(shape: Shape, cfg: int = 0, sys_id: int = 0, chol_scale: float = 1.0):
    """Return (eps[n], chol[Q][n][n]) drawn with the recipe in the module docstring."""
    o, v, nq = shape.o, shape.v, shape.nchol
    n = o + v
    rng = rng_for(cfg, sys_id)
    occ = np.sort(rng.uniform(-2.0, -0.3, size=o - 1))
    vir = np.sort(rng.uniform(0.1, 3.0, size=v))
    eps = np.concatenate([[CORE_EPS], occ, vir]).astype(np.float64)
    iu = np.triu_indices(n)
    chol = np.empty((nq, n, n), dtype=np.float64)
    for q in range(nq):
        vals = rng.standard_normal(iu[0].size) * (0.1 * np.exp(-q / 16.0) * chol_scale)
        m = np.zeros((n, n))
        m[iu] = vals
        m = m + np.triu(m, 1).T
        chol[q] = m
    return eps, chol


def draw_amplitudes(rng: np.random.Generator, shapes: dict, sigma: float):
    """Complex N(0, sigma^2) arrays for each named shape, in the dict's order."""
    out = {}
    for name, shp in shapes.items():
        re = rng.standard_normal(shp) * sigma
        im = rng.standard_normal(shp) * sigma
        out[name] = re + 1j * im
    return out


def batched_shapes(n_sys: int = 16, cfg: int = 2):
    """Uneven shapes for the batched workload: o in [5,20], v in [40,200], Q = 4 v."""
    rng = rng_for(cfg, 10_000)
    shapes = []
    for _ in range(n_sys):
        o = int(rng.integers(5, 21))
        v = int(rng.integers(40, 201))
        shapes.append(Shape(o=o, v=v, nchol=4 * v))
    return shapes
