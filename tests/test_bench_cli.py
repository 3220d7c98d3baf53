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


def test_per_workload_defaults():
    """Restarts past the residual plateau where FGMRES(30) stalls (cfg2's shear
    layer, Re = S = 1000), all-FP64 at Re = S = 1000; explicit options win."""
    a = bench.parse_args([])
    assert (a.config, a.restart, a.maxit, a.precision, a.orth) == ("cfg3", 30, 1000, "fp32", "auto")
    a = bench.parse_args(["--config", "cfg2"])
    assert (a.restart, a.maxit, a.precision) == (1000, 3000, "fp32")
    a = bench.parse_args(["--config", "cfg3_re1000"])
    assert (a.restart, a.maxit, a.precision) == (2000, 2500, "fp64")
    a = bench.parse_args(["--config", "cfg3_re1000", "--precision", "fp32", "--restart", "500"])
    assert (a.restart, a.precision) == (500, "fp32")
    assert bench.orth_name("auto", 30, 5_718_656).endswith("delayed reorthogonalisation")
    assert bench.orth_name("auto", 30, 5288) == "CGS2"
    assert bench.orth_name("auto", 2000, 5288).endswith("delayed reorthogonalisation")


def test_reported_traffic_is_the_committed_counter_summary():
    """The J traffic bench.py reports is the calibrated FETCH_SIZE + WRITE_SIZE
    figure of the committed rocprofv3 summary."""
    text = open(os.path.join(REPO, "profiles", "pmc_cfg3_jacobian_fetch_write.md")).read()
    m = re.search(r"calibrated traffic per launch \| ([0-9.]+) GB", text)
    assert m, "traffic line missing from the counter summary"
    assert abs(float(m.group(1)) * 1e9 - bench.JAC_COUNTERS["traffic_bytes"]) <= 1e6
    assert bench.JAC_COUNTERS["config"] == "cfg3"


def test_reported_sweep_traffic_and_duration_are_the_committed_summaries():
    """The paired sweep step's traffic and rocprofv3 duration that bench.py uses
    are those of the committed summaries, for the kernel source they measured."""
    text = open(os.path.join(REPO, "profiles", "pmc_cfg3_sweep_step_fetch_write.md")).read()
    m = re.search(r"calibrated traffic per launch \| \*\*([0-9.]+) MB\*\*", text)
    assert m, "traffic line missing from the sweep counter summary"
    assert abs(float(m.group(1)) * 1e6 - bench.SWEEP_COUNTERS["traffic_bytes"]) <= 1e4
    d = re.search(r"`bench.sweep_kernel_digest\(\)`\): `([0-9a-f]{16})`", text)
    assert d and d.group(1) == bench.SWEEP_COUNTERS["source_sha256_16"]
    stats = open(os.path.join(REPO, "profiles", "kstats_cfg3_fgmres_fp32_pipeline.md")).read()
    row = re.search(r"BodyStCheb<float>, st::BodyStCheb<float> >.*?\| (\d+) \| ([0-9.]+) \| ([0-9.]+) \|", stats)
    assert row and abs(float(row.group(3)) - bench.SWEEP_ROCPROF["avg_us"]) <= 0.005
    assert bench.SWEEP_ROCPROF["source_sha256_16"] == bench.SWEEP_COUNTERS["source_sha256_16"]


def test_committed_kernel_figures_match_the_current_sources():
    """The counter and duration figures are the current kernels': their source digests match."""
    assert bench.jacobian_kernel_digest() == bench.JAC_COUNTERS["source_sha256_16"]
    assert bench.sweep_kernel_digest() == bench.SWEEP_COUNTERS["source_sha256_16"]
