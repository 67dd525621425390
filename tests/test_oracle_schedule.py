"""Pins of the oracle's operator-split sequence of hydro steps and its energy release."""
import numpy as np
import pytest

import oracle
from paper_1409_5826_amd import workloads
from tests.test_oracle_pins import DECAY


def test_one_step_schedule_is_one_batch_call():
    wl = workloads.preset("n150_r1604_arrhenius", n_zones=6)
    sched = workloads.make_schedule(wl.network, wl.zones, 1, seed=7, T_swing=0.0)
    out = oracle.integrate_schedule(wl.network, wl.zones, sched)
    ref = oracle.integrate_batch(wl.network, wl.zones)
    for key in ("Y", "dt", "n_acc", "n_rej", "status"):
        np.testing.assert_array_equal(out[key], ref[key])


def test_energy_of_a_decay_is_the_product_gain():
    """A -> B with q = (0, 1): the energy of each step is the abundance B gained in it, and
    the steps' energies add up to the total gain (telescoping) to rounding."""
    zones = workloads.Zones(Y0=np.array([[1.0, 0.0]]), t_end=np.array([1.0]),
                            dt0=np.array([1e-6]), k=np.array([[2.0]]))
    sched = workloads.Schedule(T=None, dt_hydro=np.full((5, 1), 0.2), q=np.array([0.0, 1.0]))
    out = oracle.integrate_schedule(DECAY, zones, sched)
    assert out["status"][0] == oracle.ZONE_OK
    assert out["energy"].sum() == pytest.approx(out["Y"][0, 1], rel=1e-14)
    # every step releases the B created in it: e^{-2 t} decays, so does the release
    e = out["energy"][:, 0]
    assert np.all(np.diff(e) < 0) and e[0] == pytest.approx(1 - np.exp(-0.4), rel=0.05)


def test_energy_telescopes_on_a_network():
    wl = workloads.preset("n16_r48_const", n_zones=3)
    sched = workloads.make_schedule(wl.network, wl.zones, 4, seed=3)
    out = oracle.integrate_schedule(wl.network, wl.zones, sched)
    total = (out["Y"] - wl.zones.Y0) @ sched.q
    np.testing.assert_allclose(out["energy"].sum(axis=0), total, rtol=1e-12,
                               atol=1e-12 * np.abs(sched.q).max())


def test_split_steps_carry_the_trial_step():
    """Two half intervals with the trial step carried approximate the whole interval: the
    clipping at the midpoint changes the step sequence only slightly (same rates)."""
    wl = workloads.preset("n16_r48_const", n_zones=2)
    sched = workloads.make_schedule(wl.network, wl.zones, 2, seed=1)
    split = oracle.integrate_schedule(wl.network, wl.zones, sched)
    whole = oracle.integrate_batch(wl.network, wl.zones)
    assert np.all(np.abs(split["n_acc"] - whole["n_acc"]) <= 0.02 * whole["n_acc"] + 2)
    big = whole["Y"] > 1e-6
    assert np.max(np.abs(split["Y"] - whole["Y"])[big] / whole["Y"][big]) < 0.05


def test_first_failure_is_kept():
    """A zone that fails in one step keeps that status even if later steps succeed."""
    zones = workloads.Zones(Y0=np.array([[1.0, 0.0], [1.0, 0.0]]), t_end=np.array([1.0, 1.0]),
                            dt0=np.array([1e-3, 1e-3]), k=np.array([[1.0], [1.0]]))
    sched = workloads.Schedule(T=None, dt_hydro=np.array([[0.5, 0.5], [0.5, 0.5]]),
                               q=np.zeros(2))
    out = oracle.integrate_schedule(DECAY, zones, sched, opts=oracle.options(max_steps=300))
    assert (out["status"] == oracle.ZONE_MAX_STEPS).all()
    assert (out["n_acc"] + out["n_rej"] == 600).all()
