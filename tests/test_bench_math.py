"""Host-side arithmetic of bench.py (no GPU): the solve-level roofline."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_solve_roofline_sums_the_binding_bound_of_each_class():
    # 1 ms of FP32 matrix work, 1 ms of HBM traffic, and a class bound by neither alone
    stats = {"factor": {"launches": 3, "ms": 5.0, "flops": bench.FP32_PEAK_TFLOPS * 1e9, "bytes": 0.0},
             "block_solve": {"launches": 7, "ms": 2.0, "flops": 1e6, "bytes": bench.HBM_PEAK_GBS * 1e6},
             "gmres_ortho": {"launches": 2, "ms": 1.0, "flops": bench.FP64_PEAK_TFLOPS * 0.5e9,
                             "bytes": bench.HBM_PEAK_GBS * 0.25e6},
             "prolong": {"launches": 0, "ms": 0.0, "flops": 1e30, "bytes": 1e30}}
    r = bench.solve_roofline(stats, True, 5.0)
    assert r["bound_ms"] == pytest.approx(1.0 + 1.0 + 0.5)
    assert r["frac"] == pytest.approx(2.5 / 5.0)
    # FP64 factors: the factorisation is priced at the FP64 matrix peak
    r64 = bench.solve_roofline(stats, False, 5.0)
    assert r64["bound_ms"] == pytest.approx(bench.FP32_PEAK_TFLOPS / bench.FP64_PEAK_TFLOPS + 1.5)
