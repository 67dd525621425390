"""Host-side checks of the benchmark script (no GPU)."""
import os
import subprocess
import sys

import bench
from paper_1409_5826_amd import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_multi_gpu_request_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2 and "one GPU" in res.stderr


def test_algorithmic_bytes():
    net = workloads.preset("n150_r1604_arrhenius", n_zones=1).network
    assert (net.n_reactions, net.n_destruction, net.n_species) == (1604, 2727, 150)
    assert bench.algorithmic_bytes_per_zone_step(150, 1604, 2727) == 118606
    assert bench.LDS_PEAK_GBS == 256 * 128 * 2.4


def test_profiled_traffic_tied_to_sources():
    t = bench.profiled_traffic("n150_r1604_arrhenius")
    assert t is None or t > 0
    assert bench.profiled_traffic("no_such_workload") is None
