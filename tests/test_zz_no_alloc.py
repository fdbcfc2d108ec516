"""rteom_spectral_noalloc (the entry point for callers that cannot allocate device memory)
against rteom_spectral, through the C ABI on cuda:0: two calls in a row on the same
context, the second with a smaller input (fewer frequencies, and a longer history in
between), each equal bitwise to the allocating entry point (the same kernels on the same
data); sizes beyond the fixed array are refused before any device work."""
import numpy as np
import pytest

from paper_2301_04249_amd import rteom
from synthetic import TINY, draw_system

pytestmark = pytest.mark.gpu


def test_spectral_noalloc_matches_allocating_entry_point():
    eps, chol = draw_system(TINY, cfg=0)
    P = rteom.Propagator(eps, chol, 4, 4, 0, 1, workspace="torch", fixed_iters=3)
    P.step(0.025, 60)
    grids = (np.arange(-26.0, -14.0, 0.001), np.arange(-21.0, -19.0, 0.004))
    for k, omegas in enumerate(grids):
        a_ref, qp_ref, amax_ref = P.spectral(omegas, 0.01, e_corr=0.05 * k)
        a, qp, amax = P.spectral(omegas, 0.01, e_corr=0.05 * k, noalloc=True)
        print(f"call {k}: n_w={omegas.size}, steps={len(P.cumulant()[0]) - 1}, QP {qp:.9f} Eh", flush=True)
        assert np.array_equal(a, a_ref)
        assert qp == qp_ref and amax == amax_ref
        assert np.isfinite(a).all() and np.abs(a).max() > 0
        P.step(0.025, 7)
    too_many = np.linspace(-21.0, -19.0, 2_100_000)      # 2 n_w alone exceeds 4194304 doubles
    with pytest.raises(rteom.RteomError) as ex:
        P.spectral(too_many, 0.01, noalloc=True)
    assert ex.value.status == 1 and "fixed scratch" in str(ex.value)
    P.close()
