"""Host-side pieces of bench.py: the byte model and the oracle's per-routine split."""
import os
import sys

import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def test_cpu_routines_cover_the_oracle_step():
    r = bench.cpu_routines(24, (1, 1))
    assert set(r) == {"convdiff", "BDIM", "BC", "project", "CFL", "step"}
    parts = r["convdiff"] + r["BDIM"] + r["BC"] + r["project"] + r["CFL"]
    # the TGV has no body: the oracle never calls its BDIM blend
    assert r["BDIM"] == 0.0
    assert r["convdiff"] > 0 and r["project"] > 0 and r["CFL"] > 0
    # the timed routines are disjoint parts of the step
    assert parts <= r["step"] * 1.0001


def test_cpu_baseline_reports_the_oracle():
    r = bench.cpu_baseline(24, (1, 1))
    assert r["kind"] == "oracle" and r["cores"] == 1 and r["value"] > 0


@pytest.mark.parametrize("fused", [False, True])
def test_step_bytes_grow_with_vcycles(fused):
    assert bench.step_bytes_per_cell(2, fused) > bench.step_bytes_per_cell(0, fused) > 0
