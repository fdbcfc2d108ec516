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


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("fp32", 1e-5), ("bf16x3", 1e-3), ("fp16x3", 1e-5)])
def test_esca_embedded_parity(emb, prec, tol):
    print(f"ESCA-shaped residual, prec={prec}", flush=True)
    P = rteom.Propagator(emb["eps"], emb["chol"], ESCA_PAPER.o, ESCA_PAPER.o, 0, 1, prec=prec, fixed_iters=2,
                         workspace="torch")
    try:
        embedding.check(P, emb, prec, tol)
    finally:
        P.close()


def test_esca_contract_shape_embedded_parity(capsys):
    """The benchmark's own shape and launch configuration: o=71, v=649 per spin (beta hole),
    Q=2000, float64, one fixed-point pass, the memory plan bench.py runs (integral slabs
    rebuilt per residual, blocked ring intermediates).  The tiny system is embedded as a
    non-interacting part (tests/embedding.py); amplitudes are written and the residual is read
    in device memory.  Its residual block matches the oracle element by element, every
    element joining the parts vanishes, and the energy splits."""
    from synthetic import ESCA
    print(f"drawing the ESCA-shaped system o={ESCA.o} v={ESCA.v} Q={ESCA.nchol}", flush=True)
    emb = embedding.build(ESCA, 4, TINY.o, TINY.v, TINY.nchol)
    P = rteom.Propagator(emb["eps"], emb["chol"], ESCA.o, ESCA.o, 0, 1, prec="fp64", fixed_iters=1,
                         tune=False, workspace="torch", max_steps=4, progress=True)
    del emb["chol"]
    plan = P.plan()
    print(f"plan {plan}", flush=True)
    assert not plan["resident"]

    def run(fn):
        with capsys.disabled():     # the library's progress lines (one per block) reach the log
            fn()

    try:
        err, mixed, e_err = embedding.check_device(P, emb, 1e-11, run)
    finally:
        P.close()
    assert err < 1e-11
    assert mixed <= 1e-13
    assert e_err <= 1e-11


def test_zn_porphyrin_shape_embedded_parity(capsys):
    """The Zn-porphyrin shape: o=95, v=560 per spin (beta hole: 95/94 occupied, 560/561
    virtual), Q=3000, fp16x3 contractions with float64 update, one fixed-point pass (two
    amplitude sets: no right-hand-side set), integral slabs rebuilt per residual.  The tiny
    system is embedded as a non-interacting part: its residual block against the oracle,
    every element joining the parts zero, and the energy split."""
    from synthetic import ZN_PORPHYRIN as ZN
    print(f"drawing the Zn-porphyrin-shaped system o={ZN.o} v={ZN.v} Q={ZN.nchol}", flush=True)
    emb = embedding.build(ZN, 5, TINY.o, TINY.v, TINY.nchol)
    P = rteom.Propagator(emb["eps"], emb["chol"], ZN.o, ZN.o, 0, 1, prec="fp16x3", fixed_iters=1,
                         tune=False, workspace="torch", max_steps=4, progress=True)
    del emb["chol"]
    plan = P.plan()
    print(f"plan {plan}", flush=True)
    assert not plan["resident"]

    def run(fn):
        with capsys.disabled():
            fn()

    try:
        err, mixed, e_err = embedding.check_device(P, emb, 1e-5, run)
    finally:
        P.close()
    assert err < 1e-5
    assert mixed <= 1e-12
    assert e_err <= 1e-11
