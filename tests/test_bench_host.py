"""Host logic of bench.py (CPU): the one-GPU guard and the reading of the
committed counter summary, which must be dropped once the kernel source it was
taken on has changed."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_counter_summary_is_tied_to_the_kernel_source(monkeypatch):
    vals = bench.spmm_counters("mixed", 8)
    if vals is None:
        pytest.skip("counter summary taken on another version of the kernel source")
    hbm = bench.spmm_traffic("mixed", 8)
    assert hbm == float(vals["hbm_bytes_per_launch"]) > 0
    fill = bench.spmm_l2_fill("mixed", 8, 0.025)
    assert fill["bytes"] == float(vals["l2_to_l1_bytes_per_launch"])
    assert fill["achieved"] == pytest.approx(fill["bytes"] / 0.025e-3 / 1e9, abs=0.06)
    assert fill["peak"] == pytest.approx(8 * 16 * 128 * 2.4)
    assert bench.spmm_l2_fill("mixed", 8, 0.0) is None
    monkeypatch.setattr(bench, "_source_hash", lambda: "0" * 16)
    assert bench.spmm_traffic("mixed", 8) is None
    assert bench.spmm_l2_fill("mixed", 8, 0.025) is None
    # no summary for a width that was never measured
    monkeypatch.undo()
    assert bench.spmm_traffic("mixed", 32) is None
