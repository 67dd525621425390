"""Calibrate the activation-energy windows of the Arrhenius workloads.

Runs only the CPU oracle on the generated zones and prints, for each
candidate window E ~ U(E_lo, E_hi), the 10th/50th/90th percentiles of the
accepted step counts and their p90/p10 spread.  The windows frozen in
paper_1409_5826_amd/workloads.py are the ones whose spread is about 10x.

    python tests/calibrate_arrhenius.py
"""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import oracle  # noqa: E402
from paper_1409_5826_amd import workloads  # noqa: E402


def spread(name, n_zones, window):
    wl = workloads.preset(name, n_zones=n_zones, e_window=window)
    out = oracle.integrate_batch(wl.network, wl.zones)
    p10, p50, p90 = np.percentile(out["n_acc"], [10, 50, 90])
    return p10, p50, p90, p90 / p10


def main():
    for name, n_zones, lows in [("n150_r1604_arrhenius", 128, (0.0, 26.0, 27.5, 29.0)),
                                ("n365_r4400_arrhenius", 64, (0.0, 28.0, 30.0, 31.0))]:
        for lo in lows:
            p10, p50, p90, ratio = spread(name, n_zones, (lo, 90.0))
            print(f"{name} E~U({lo:g},90): p10 {p10:.0f} p50 {p50:.0f} p90 {p90:.0f} "
                  f"p90/p10 {ratio:.2f}", flush=True)


if __name__ == "__main__":
    main()
