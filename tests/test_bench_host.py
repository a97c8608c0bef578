"""Host logic of bench.py (no GPU): the committed traffic summaries it reads
for the roofline's `traffic`, and the refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import pytest

import bench
from paper_2411_19109_amd import profsum

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SWEEP = "yig_demux_sweep_64x_10000steps_grad"


def _record(workload):
    path = os.path.join(ROOT, "profiles", f"{workload}_hbm_traffic.txt")
    rec = None
    for line in open(path):
        if line.startswith("{"):
            rec = json.loads(line)
    return rec


def test_committed_traffic_summary_is_read_for_its_kernel_source():
    rec = _record(SWEEP)
    if rec["kernel_source_sha256"] != profsum.kernel_source_hash("llg_kernels.hip"):
        pytest.skip("the traffic summary was taken on another kernel source (the bench then reports null)")
    b = bench.measured_traffic(SWEEP, "k_col", rec["launch"])
    assert b is not None and b > 0
    # copy-calibrated traffic close to the column kernel's algorithmic bytes (109.6 MB per launch)
    assert 1.0 <= b / 109_587_936 <= 1.2


def test_traffic_follows_the_kernel_class_tiling_only(monkeypatch):
    rec = _record(SWEEP)
    monkeypatch.setattr(profsum, "kernel_source_hash", lambda source: rec["kernel_source_sha256"])
    launch = list(rec["launch"])
    other_rows = launch[:3] + [512, 16, 512, 16, 7]
    assert bench.measured_traffic(SWEEP, "k_col", other_rows) == bench.measured_traffic(SWEEP, "k_col", launch)
    other_col = [launch[0] * 2 if launch[0] < 16 else 1] + launch[1:]
    assert bench.measured_traffic(SWEEP, "k_col", other_col) is None
    # a row kernel's traffic ignores the column tiling
    assert bench.measured_traffic(SWEEP, "k_stage_fwd", other_col) == bench.measured_traffic(SWEEP, "k_stage_fwd", launch)


def test_traffic_is_none_without_a_summary_or_on_another_source(monkeypatch):
    assert bench.measured_traffic("no_such_workload", "k_col", [1] * 8) is None
    monkeypatch.setattr(profsum, "kernel_source_hash", lambda source: "0" * 64)
    assert bench.measured_traffic(SWEEP, "k_col", _record(SWEEP)["launch"]) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "GPU" in (r.stdout + r.stderr)
