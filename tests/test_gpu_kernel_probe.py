"""GEMM and permute kernels of the library, case by case (tests/kernel_probe/kernel_probe.cpp):
every operand layout, complex combination, ragged size, split-K factor, broadcast batch and
tile shape against host loops in float64 (1e-12), float32 (2e-5), bf16x3 (2e-3) and fp16x3
(1e-5 of the sum of magnitudes, rows and columns scaled over 2^-20..2^20); tile
shapes and the converted-operand paths bitwise equal to the 64x64 result; permutes against
host loops (1e-14); pair storage pack/unpack against host loops written from the definition."""
import os
import subprocess

import pytest

pytestmark = pytest.mark.gpu

PROBE = os.path.join(os.path.dirname(__file__), "kernel_probe", "kernel_probe")


def test_kernel_probe():
    if not os.path.exists(PROBE):
        pytest.fail("kernel probe not built (run __graft_entry__.build())")
    out = subprocess.run([PROBE], capture_output=True, text=True, timeout=600)
    print(out.stdout[-4000:])
    assert "permute probe:" in out.stdout and "gemm probe:" in out.stdout
    assert " 0 failures" in out.stdout.split("permute probe:")[1].splitlines()[0]
    assert " 0 failures" in out.stdout.split("gemm probe:")[1].splitlines()[0]
    assert "pairs probe:" in out.stdout
    assert " 0 failures" in out.stdout.split("pairs probe:")[1].splitlines()[0]
    assert out.returncode == 0
