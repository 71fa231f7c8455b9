"""CPU checks of the benchmark's host logic (no GPU needed)."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_algorithmic_bytes_per_unit_figures():
    # one RHS: 10 outer iterations, sum of active shifts 30, 40 inner iterations, M = 64, 100 block entries
    stats = np.array([[10, 30, 40, 0, 64, 100, 0, 0]], dtype=np.int64)
    bd, K, nout = 4, 8, np.array([12])
    blk = 100 * bd * bd * 8
    # projected FP64, generalized, blocks shared by 2 RHS
    got = bench.algorithmic_bytes(stats, nout, K, bd, True, 0, True, 2, True)
    want = (30 * 12 * 4 * 16 + 10 * 12 * 16) + 10 * (2 * blk / 2 + 2 * 16 * 64) + 40 * (blk / 2 + 6 * 16 * 64)
    assert np.isclose(got, want)
    # full x, S = I, FP32 vectors and blocks, audit: one operator pass per shift
    got = bench.algorithmic_bytes(stats, nout, K, bd, False, 1, False, 1, True)
    blk4 = 100 * bd * bd * 4
    want = (30 * 64 * 4 * 8 + 10 * 64 * 8) + 10 * (blk4 + 2 * 8 * 64) + K * (100 * bd * bd * 8 + 32 * 64)
    assert np.isclose(got, want)


def test_workloads_name_their_configurations():
    assert set(bench.WORKLOADS) >= {"cfg0", "cfg1", "cfg2", "cfg2r", "cfg4r"}
    assert bench.WORKLOADS["cfg2r"]["radius"] == (1.0, 2.0)
