"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the workload table and the
per-precision tables it reports from, and the profile summaries its traffic figures cite."""
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from synthetic import ESCA, ZN_PORPHYRIN  # noqa: E402


def test_more_than_one_gpu_is_refused(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err


def test_precision_tables_cover_every_choice():
    precs = {"fp64", "fp32", "bf16x3", "fp16x3"}
    for table in (bench.KERNEL_NAME, bench.DTYPE, bench.EXEC_PER_USEFUL, bench.RATE_GUESS, bench.PEAK_TFLOPS):
        assert set(table) == precs
    # the split precisions execute three 16-bit products per useful one, against the 16-bit peak
    assert bench.EXEC_PER_USEFUL["bf16x3"] == bench.EXEC_PER_USEFUL["fp16x3"] == 3.0
    assert bench.PEAK_TFLOPS["fp64"] == 78.6 and bench.PEAK_TFLOPS["fp32"] == 157.3


def test_workloads():
    w = bench.WORKLOADS
    assert w["esca"]["shape"] == ESCA and w["esca"]["passes"] == 1 and w["esca"]["large"]
    assert w["zn"]["shape"] == ZN_PORPHYRIN and w["zn"]["passes"] == 1 and w["zn"]["large"]
    for name, work in w.items():
        assert work["desc"], name
        if work.get("large"):
            # every large workload has a bounded CPU baseline: a restricted slab or a small system
            assert work.get("cpu_slab_vir") or not w[work["cpu_sample"]].get("large"), name
    assert bench.chol_scale(ESCA) == pytest.approx((16.0 / ESCA.v) ** 0.5)


def test_traffic_figures_cite_committed_profiles():
    for (workload, prec), (value, source) in bench.TRAFFIC.items():
        assert workload in bench.WORKLOADS and value > 0
        path = source.split(":")[0].split(" ")[0]
        assert os.path.exists(os.path.join(ROOT, path)), source
