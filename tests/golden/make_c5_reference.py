"""Write c5_radau_reference.json: converged final abundances of the zones on which the
learned-vs-plain comparison measures its final-abundance error.

The zones are the first 256 of the 4096 held-out zones of the 150-species constant-rate
workload (workloads.preset("n150_r1604_const", n_zones=4096, seed_offset=1003)); each is
integrated over its interval by oracle.ode_reference.radau (scipy Radau IIA, rtol 1e-9,
atol 1e-20, analytic sparse Jacobian; abundances below 1e-20 weigh nothing in the mass-fraction
error, and tighter settings take up to hours for some zones).  Zones 0 and 3 are also
integrated at rtol 1e-10; the larger mass-fraction L1 difference of the two solutions is stored
as the reference's error estimate.  Calls only the oracle and the seeded input generator.

    python tests/golden/make_c5_reference.py
"""
import json
import os
import sys
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import ode_reference  # noqa: E402
from paper_1409_5826_amd import workloads  # noqa: E402

N_ZONES = 256
RTOL, ATOL = 1e-9, 1e-20
CHECK_ZONES = (0, 3)
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_radau_reference.json")


def _wl():
    return workloads.preset("n150_r1604_const", n_zones=4096, seed_offset=1003)


def _solve(args):
    import time

    z, rtol = args
    wl = _wl()
    t0 = time.perf_counter()
    Y, nfev, nsteps = ode_reference.radau(wl.network, wl.zones.k[z], wl.zones.Y0[z],
                                          wl.zones.t_end[z], rtol=rtol, atol=ATOL)
    print(f"zone {z} rtol {rtol:g}: {nsteps} steps, {nfev} evaluations, "
          f"{time.perf_counter() - t0:.0f} s", flush=True)
    return z, rtol, Y, nfev, nsteps


def main():
    wl = _wl()
    w = wl.network.weight.astype(np.float64)
    jobs = [(z, RTOL / 10) for z in CHECK_ZONES] + [(z, RTOL) for z in range(N_ZONES)]
    with Pool(min(8, os.cpu_count() or 1)) as pool:
        res = list(pool.imap_unordered(_solve, jobs))
    Y = np.zeros((N_ZONES, wl.network.n_species))
    tight = {}
    for z, rtol, y, _, _ in res:
        if rtol == RTOL:
            Y[z] = y
        else:
            tight[z] = y
    est = max(float(w @ np.abs(tight[z] - Y[z])) for z in tight)
    doc = {
        "what": f"Y(t_end) of Eq. (eq1.1) by scipy Radau for zones 0..{N_ZONES - 1} of "
                "n150_r1604_const (4096 zones, seed_offset 1003)",
        "workload": "n150_r1604_const", "n_zones_total": 4096, "seed_offset": 1003,
        "zones": list(range(N_ZONES)), "rtol": RTOL, "atol": ATOL,
        "error_estimate_mass_fraction_l1": est,
        "Y": [[float(v) for v in row] for row in Y],
    }
    with open(OUT, "w") as fh:
        json.dump(doc, fh)
    print(f"wrote {OUT}: {N_ZONES} zones, reference error estimate {est:.2e}")


if __name__ == "__main__":
    main()
