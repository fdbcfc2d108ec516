"""T2 amplitude storage of Table 2.

Sec. 2.3: with spin-integrated equations only the alpha-alpha, beta-beta and
alpha-beta doubles blocks are stored, and the update of Eq. trapzrule keeps
three such "timeline" tensors.  Table 2 lists the per-tensor size; it is
reproduced by full (unpacked) complex128 blocks counted in GiB.
"""
from __future__ import annotations

BYTES_COMPLEX128 = 16


def t2_bytes(no_a: int, no_b: int, nv_a: int, nv_b: int, bytes_per=BYTES_COMPLEX128) -> int:
    """Bytes of one T2 tensor: full aa + bb + ab blocks."""
    aa = no_a * no_a * nv_a * nv_a
    bb = no_b * no_b * nv_b * nv_b
    ab = no_a * no_b * nv_a * nv_b
    return (aa + bb + ab) * bytes_per


def t2_gib(no_a: int, no_b: int, nv_a: int, nv_b: int) -> float:
    return t2_bytes(no_a, no_b, nv_a, nv_b) / 2.0 ** 30


# Table 2 rows: (n_occ_alpha, n_occ_beta, n_vir_alpha, n_vir_beta, T2 GB per tensor)
TABLE2 = {
    "Uracil": (29, 28, 351, 352, 4.5),
    "ESCA": (36, 35, 404, 405, 9.2),
    "Benzene-Ammonia": (26, 25, 444, 445, 5.8),
    "Zn-porphyrin": (95, 94, 1130, 1131, 510.2),
}
