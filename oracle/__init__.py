"""CPU oracle for the RT-EOM-CCSD hot path (arXiv 2301.04249).

TEST INFRASTRUCTURE ONLY.  Plain, slow, float64/complex128 NumPy code that
states what the GPU path must compute.  Only the tests, the smoke entry point
and the benchmark's CPU-baseline leg may import it; the library never does,
and it shares no code with the library (only the seeded input generator in
``synthetic`` serves both).

Modules
-------
reference   spin-orbital (N-1)-electron reference, Fock matrix and
            antisymmetrised integrals (Sec. 2.1, the Fock definition next to
            the normal-ordered Hamiltonian; Sec. 2.3 for the Cholesky form).
ccsd        the CCSD amplitude residual (Eqs. dt1eom/dt2eom) and the cumulant
            derivative functional (Eq. cum_gf3 / Eq. dcdt).
propagate   implicit trapezoidal (first-order Adams-Moulton) step with
            fixed-point micro-iterations (Eq. trapzrule), C(t), G(t) and
            A(omega) (Eqs. cum_gf, cum_gf2).
fockspace   brute-force determinant-space evaluation of the projections that
            define the residual and the energy (pins the ccsd module), and
            the exact propagation <Phi|exp(i H_N t)|Phi> by diagonalisation
            (pins the integrator where CCSD is exact: two electrons).
memory      the T2 storage formula of Table 2.

Parity status: every function here is pinned by a test in tests/ against
brute force, closed forms or the paper's Table 2, except where its docstring
says "parity unpinned".
"""
