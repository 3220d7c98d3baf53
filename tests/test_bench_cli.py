"""bench.py's command-line contract and the consistency of its committed
hardware-counter figure (host only)."""
import os
import re
import subprocess
import sys

import bench

REPO = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(REPO, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=REPO)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_reported_traffic_is_the_committed_counter_summary():
    """The J traffic bench.py reports is the calibrated FETCH_SIZE + WRITE_SIZE
    figure of the committed rocprofv3 summary."""
    text = open(os.path.join(REPO, "profiles", "pmc_cfg3_jacobian_fetch_write.md")).read()
    m = re.search(r"calibrated traffic per launch \| ([0-9.]+) GB", text)
    assert m, "traffic line missing from the counter summary"
    assert abs(float(m.group(1)) * 1e9 - bench.JAC_COUNTERS["traffic_bytes"]) <= 1e6
    assert bench.JAC_COUNTERS["config"] == "cfg3"
