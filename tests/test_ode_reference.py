"""Pins of the converged ODE reference (oracle/ode_reference.py): closed forms the scipy
Radau solution must reproduce, independent of the explicit integrator."""
import numpy as np
import scipy.linalg

from oracle import ode_reference
from paper_1409_5826_amd import workloads


class _Net:
    def __init__(self, n, r0, r1, pr, w=None):
        self.n_species = n
        self.reactant0 = np.asarray(r0)
        self.reactant1 = np.asarray(r1)
        self.product = np.asarray(pr)
        self.weight = None if w is None else np.asarray(w)


def test_linear_network_matches_matrix_exponential():
    """One-body reactions only: dY/dt = A Y, Y(t) = expm(A t) Y0 (a different algorithm)."""
    rng = np.random.default_rng(3)
    n = 6
    r0 = [0, 1, 2, 3, 4, 5, 0, 2, 4]
    pr = [1, 2, 3, 4, 5, 0, 3, 5, 1]
    k = 10.0 ** rng.uniform(-1, 3, size=len(r0))
    net = _Net(n, r0, [-1] * len(r0), pr)
    A = np.zeros((n, n))
    for j, (a, c) in enumerate(zip(r0, pr)):
        A[a, a] -= k[j]
        A[c, a] += k[j]
    Y0 = rng.dirichlet(np.ones(n))
    Y, _, _ = ode_reference.radau(net, k, Y0, 0.05)
    want = scipy.linalg.expm(A * 0.05) @ Y0
    np.testing.assert_allclose(Y, want, rtol=1e-8, atol=1e-14)


def test_two_body_closed_form():
    """A + B -> C:  Y_A(t) = D Y_A0 / (Y_B0 e^{k D t} - Y_A0) with D = Y_B0 - Y_A0."""
    net = _Net(3, [0], [1], [2], w=[1, 1, 2])
    k, ya, yb = 37.0, 0.3, 0.5
    t = 0.2
    Y, _, _ = ode_reference.radau(net, [k], [ya, yb, 0.0], t)
    d = yb - ya
    want_a = d * ya / (yb * np.exp(k * d * t) - ya)
    np.testing.assert_allclose(Y[0], want_a, rtol=1e-8)
    np.testing.assert_allclose(Y[1], want_a + d, rtol=1e-8)
    np.testing.assert_allclose(Y[2], ya - want_a, rtol=1e-8)


def test_weighted_sum_conserved_on_a_stiff_network():
    """The exact ODE conserves sum w Y (each reaction conserves weight); the reference keeps
    it to its tolerance on a stiff 16-species network with rates over 12 decades."""
    wl = workloads.preset("n16_r48_const", n_zones=1)
    net, z = wl.network, wl.zones
    Y, _, _ = ode_reference.radau(net, z.k[0], z.Y0[0], z.t_end[0])
    w = net.weight.astype(float)
    assert abs(w @ Y - w @ z.Y0[0]) <= 1e-9 * (w @ z.Y0[0])
    assert (Y > -1e-12).all()


def test_committed_c5_reference_is_consistent():
    """The stored reference (tests/golden/c5_radau_reference.json): one row per listed zone,
    finite and non-negative to the absolute tolerance, Σ w Y(t_end) equal to Σ w Y(0) (a linear invariant of Eq. eq1.1
    that Radau keeps to its tolerance), and the fastest zone re-solved by the generator's own
    call reproduces its row within the stored error estimate."""
    import json
    import os
    import time

    path = os.path.join(os.path.dirname(__file__), "golden", "c5_radau_reference.json")
    with open(path) as fh:
        ref = json.load(fh)
    wl = workloads.preset(ref["workload"], n_zones=ref["n_zones_total"],
                          seed_offset=ref["seed_offset"])
    zones = np.asarray(ref["zones"])
    Y = np.asarray(ref["Y"])
    assert Y.shape == (len(zones), wl.network.n_species) and len(zones) >= 256
    # Radau keeps abundances non-negative only to its absolute tolerance
    assert np.isfinite(Y).all() and (Y >= -10 * ref["atol"]).all()
    w = wl.network.weight.astype(np.float64)
    m0 = wl.zones.Y0[zones] @ w
    assert np.abs(Y @ w - m0).max() <= 1e-7 * m0.max()
    # zone 0 and 3 were also solved 10x tighter; re-solve one zone here (a few seconds)
    z = 128
    t0 = time.perf_counter()
    Yz, _, _ = ode_reference.radau(wl.network, wl.zones.k[z], wl.zones.Y0[z], wl.zones.t_end[z],
                                   rtol=ref["rtol"], atol=ref["atol"])
    assert time.perf_counter() - t0 < 120
    assert w @ np.abs(Yz - Y[list(zones).index(z)]) <= max(ref["error_estimate_mass_fraction_l1"],
                                                           1e-12)
