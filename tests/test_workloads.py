"""Checks of the seeded workload generator (host only)."""
import numpy as np
import pytest

from paper_1409_5826_amd import workloads

SIZES = {
    "n16_r48_const": (16, 24, 24),
    "n150_r1604_const": (150, 481, 1123),
    "n150_r1604_arrhenius": (150, 481, 1123),
    "n365_r4400_arrhenius": (365, 1320, 3080),
}


@pytest.mark.parametrize("name", sorted(SIZES))
def test_network_structure(name):
    wl = workloads.preset(name, n_zones=3)
    net = wl.network
    n, r1, r2 = SIZES[name]
    assert net.n_species == n and net.n_one_body == r1 and net.n_two_body == r2
    a, b, c, w = net.reactant0, net.reactant1, net.product, net.weight
    assert a.min() >= 0 and a.max() < n and c.min() >= 0 and c.max() < n
    assert b.max() < n and (b[b < 0] == -1).all()
    two = b >= 0
    assert (a != b).all() and (c != a).all() and (c[two] != b[two]).all()
    # every reaction conserves weight (Eq. 5.35 with integer mass numbers)
    assert (w[c[~two]] == w[a[~two]]).all()
    assert (w[c[two]] == w[a[two]] + w[b[two]]).all()
    # no duplicate reaction (unordered reactants)
    keys = {(min(x, y) if y >= 0 else x, max(x, y) if y >= 0 else -1, z)
            for x, y, z in zip(a.tolist(), b.tolist(), c.tolist())}
    assert len(keys) == net.n_reactions
    inc = np.bincount(a, minlength=n) + np.bincount(b[two], minlength=n) + np.bincount(c, minlength=n)
    assert inc.min() >= 4
    # initial abundances: sum_i w_i Y0_i = 1
    Y0 = wl.zones.Y0
    assert (Y0 >= 0).all()
    np.testing.assert_allclose(Y0 @ w, 1.0, rtol=1e-14)
    assert (wl.zones.T is None) == (net.A is None)


def test_same_seed_same_bytes():
    a = workloads.preset("n150_r1604_arrhenius", n_zones=5)
    b = workloads.preset("n150_r1604_arrhenius", n_zones=5)
    for x, y in [(a.network.reactant0, b.network.reactant0), (a.network.product, b.network.product),
                 (a.network.A, b.network.A), (a.network.E, b.network.E), (a.zones.Y0, b.zones.Y0),
                 (a.zones.T, b.zones.T)]:
        assert x.tobytes() == y.tobytes()


def test_rate_ranges():
    wl = workloads.preset("n150_r1604_const", n_zones=4)
    lk = np.log10(wl.zones.k)
    assert lk.min() >= -6 and lk.max() <= 10 and wl.zones.k.shape == (4, 1604)
    wl = workloads.preset("n150_r1604_arrhenius", n_zones=64)
    la = np.log10(wl.network.A)
    assert la.min() >= 2 and la.max() <= 12
    lo, hi = workloads.ARRHENIUS_E_WINDOW_N150
    assert wl.network.E.min() >= lo and wl.network.E.max() <= hi
    assert wl.zones.T.min() >= 1 and wl.zones.T.max() <= 4
