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
    # rates held in registers (the packed-rows kernel): one value per reaction less
    assert bench.algorithmic_bytes_per_zone_step(150, 1604, 2727) == 105774
    assert bench.algorithmic_bytes_per_zone_step(150, 1604, 2727, 8, False) == 118606
    assert bench.algorithmic_bytes_per_zone_step(365, 4400, 7480) == 288280
    assert bench.algorithmic_bytes_per_zone_step(150, 1604, 2727, 4) == 63634 - 4 * 1604
    assert bench.LDS_PEAK_GBS == 256 * 128 * 2.4


def test_profiled_traffic_tied_to_sources():
    t = bench.profiled_traffic("n150_r1604_arrhenius")
    assert t is None or t > 0
    assert bench.profiled_traffic("no_such_workload") is None


def test_time_at_equal_error_interpolates_log_log():
    """Power laws ms = c e^-1 (plain) and 10 c e^-1 (learned) give a ratio of 10 at the
    tightest common error; disjoint error ranges give None."""
    plain = [(e, 100.0 / e) for e in (1.0, 0.3, 0.1)]
    learned = [(e, 1000.0 / e) for e in (2.0, 0.5, 0.2)]
    err, ms_p, ms_l = bench.time_at_equal_error(plain, learned)
    assert err == 0.2
    assert abs(ms_p - 500.0) < 1e-9 and abs(ms_l - 5000.0) < 1e-9
    assert bench.time_at_equal_error([(1.0, 1.0), (0.5, 2.0)], [(0.1, 5.0), (0.05, 9.0)]) is None
    # a form whose every tolerance left a reference zone unfinished has no curve
    assert bench.time_at_equal_error([(1.0, 1.0)], []) is None


def test_mass_drift_reports_the_weighted_sum_ratio():
    import numpy as np

    wl = workloads.preset("n16_r48_const", n_zones=4)
    w = wl.network.weight.astype(float)
    Y = wl.zones.Y0 * np.array([[1.0], [2.0], [0.5], [1.0]])
    d = bench.mass_drift(wl, Y)
    assert d["min"] == 0.5 and d["max"] == 2.0 and d["p50"] == 1.0
