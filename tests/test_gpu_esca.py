"""Parity at the ESCA-shaped benchmark size (o=36, v=324 per spin, Q=2000: the paper's
71 occupied / 649 virtual spin-orbitals with the beta core hole), in the launch
configuration bench.py times.  One residual there is ~4e14 flops over an 83 GiB
(ae|bf) block, far beyond the oracle, so the check embeds the tiny workload's
shape (o=4, v=16, Q=48, holding the core hole) as a non-interacting part of the
full system (tests/embedding.py): its block of the residual against the oracle,
element by element, zero elements joining the parts, antisymmetry, and the
energy split.
"""
import pytest

import embedding
from paper_2301_04249_amd import rteom
from synthetic import ESCA_PAPER, TINY

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def emb():
    print(f"drawing the ESCA-shaped system o={ESCA_PAPER.o} v={ESCA_PAPER.v} Q={ESCA_PAPER.nchol}", flush=True)
    return embedding.build(ESCA_PAPER, 3, TINY.o, TINY.v, TINY.nchol)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 1e-5), ("bf16x3", 1e-3)])
def test_esca_embedded_parity(emb, prec, tol):
    print(f"ESCA-shaped residual, prec={prec}", flush=True)
    P = rteom.Propagator(emb["eps"], emb["chol"], ESCA_PAPER.o, ESCA_PAPER.o, 0, 1, prec=prec, fixed_iters=2,
                         workspace="torch")
    try:
        embedding.check(P, emb, prec, tol)
    finally:
        P.close()
