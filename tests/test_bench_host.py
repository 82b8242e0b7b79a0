"""Host logic of bench.py, on the CPU: the algorithmic work count against the
oracle's assembled matrix, the counter-summary lookup, and the one-GPU rule."""
import os
import subprocess
import sys

import numpy as np
import pytest

import bench
from oracle import projector

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("geom", [(8, 6, 13), (12, 8, 17), (16, 10, 23), (9, 7, 14)])
def test_joseph_nnz_counts_the_matrix(geom):
    # the roofline's work per launch (2 nnz FLOP) counts the nonzero weights
    # of the Joseph matrix: the oracle's assembled matrix has exactly that many
    n, na, nd = geom
    M = projector.matrix(n, na, nd)
    assert bench.joseph_nnz(n, na, nd) == int(np.count_nonzero(M))


def test_measured_traffic_follows_the_committed_summary():
    # a line for another variant is never used; the summary's own line only
    # while the kernel sources hash as they did when the counters were taken
    assert bench.measured_traffic("project", {"fwd": 3, "adj_px": 8, "adj_shares": 6}) is None
    t = bench.measured_traffic("project", {"fwd": 4, "adj_px": -4, "adj_shares": 16})
    if t is None:
        pytest.skip("the kernel sources changed since the counter summary was taken")
    assert t > 0


def test_measured_valu_issue_follows_the_committed_summary():
    assert bench.measured_valu_issue("project", {"fwd": 3, "adj_px": 8, "adj_shares": 6}) is None
    v = bench.measured_valu_issue("backproject", {"fwd": 4, "adj_px": -4, "adj_shares": 16})
    if v is None:
        pytest.skip("the kernel sources changed since the counter summary was taken")
    frac, insts, kernel = v
    assert 0.0 < frac <= 1.0 and insts > 0 and "adj_quad" in kernel


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr


def test_cpu_baseline_legs_on_a_small_workload():
    # the oracle timed on one core (operators, one iteration) and on all
    # cores (one iteration per worker process), on the 128^2 workload
    r = bench.cpu_baseline("ellipses128_rigid4")
    assert r["kind"] == "oracle" and r["cores"] == r["all_cores"]["workers"] >= 1
    one = r["one_core"]
    assert one["s_apply_Ai"] > 0 and one["s_apply_Ai_adjoint"] > 0 and one["s_per_iteration"] > 0
    assert r["value"] == r["all_cores"]["epochs_per_s"] > 0


def test_measured_roofs_reads_the_committed_probe_summary():
    roofs = bench.measured_roofs()
    if roofs is None:
        pytest.skip("no probe summary committed")
    assert roofs["lds_read_tbs"] > 0 and roofs["copy_gbs"] > 0
