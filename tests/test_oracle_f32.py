"""Pins of the oracle's single-precision integration (state and arithmetic in float, time in
double), against closed forms, exact float arithmetic on representable values, the dense
incidence, the drift identity, the hand-traced controller and the double-precision oracle."""
import math

import numpy as np
import pytest

import oracle
from paper_1409_5826_amd import workloads
from tests.test_oracle_pins import DECAY, dense_incidence, load_trace_cases, mass_action, random_state

F32_EPS = float(np.finfo(np.float32).eps)


def test_state_is_rounded_to_float_once():
    """With zero rates nothing changes except the rounding of Y to float and back."""
    Y0 = np.array([1.0 / 3.0, 0.1])
    out = oracle.integrate_zone_f32(DECAY, np.array([0.0]), Y0, 1.0, 0.1)
    assert out["status"] == oracle.ZONE_OK
    np.testing.assert_array_equal(out["Y"], Y0.astype(np.float32).astype(np.float64))
    assert out["Y"][0] != Y0[0]


@pytest.mark.parametrize("k,h,asym", [(2.0, 0.125, False), (16.0, 0.125, True), (4.0, 0.25, True)])
def test_one_step_closed_forms_exact_in_float(k, h, asym):
    """Values representable in float with exact products: Euler (1 - k h) Y, asymptotic
    Y / (1 + k h) (k h == 1 takes the asymptotic form), the product gains h k Y."""
    Y = np.array([0.75, 0.5], dtype=np.float32)
    Fp, kd = oracle.rhs_f32(DECAY, np.array([k]), Y)
    assert Fp[0] == 0 and kd[0] == k and Fp[1] == k * 0.75 and kd[1] == 0
    Yn = oracle.update_f32(Y, Fp, kd, h)
    want = 0.75 / (1 + k * h) if asym else (1 - k * h) * 0.75
    assert Yn[0] == np.float32(want)
    assert Yn[1] == np.float32(0.5 + h * k * 0.75)


@pytest.mark.parametrize("name", ["n16_r48_const", "n150_r1604_const"])
def test_rhs_f32_matches_dense_incidence(name):
    net = workloads.preset(name, n_zones=1).network
    rng = np.random.default_rng(3)
    P, D = dense_incidence(net)
    for _ in range(3):
        k, Y = random_state(net, rng)
        k32, Y32 = k.astype(np.float32), Y.astype(np.float32)
        Fp, kd = oracle.rhs_f32(net, k32, Y32)
        f = mass_action(net, k32.astype(np.float64), Y32.astype(np.float64))
        # creation fluxes and depletion fluxes, each to float rounding of its sum
        np.testing.assert_allclose(Fp, P @ f, rtol=64 * F32_EPS, atol=1e-37)
        np.testing.assert_allclose(kd.astype(np.float64) * Y32, D @ f, rtol=64 * F32_EPS, atol=1e-37)


def test_drift_identity_in_float():
    net = workloads.preset("n16_r48_const", n_zones=1).network
    w = net.weight.astype(np.float64)
    rng = np.random.default_rng(9)
    for h in (1e-6, 1e-4, 1e-2):
        k, Y = random_state(net, rng, -2.0, 8.0)
        Y32 = Y.astype(np.float32)
        Fp, kd = oracle.rhs_f32(net, k, Y32)
        Yn = oracle.update_f32(Y32, Fp, kd, h)
        Fp, kd, Yd, Ynd = (v.astype(np.float64) for v in (Fp, kd, Y32, Yn))
        asy = kd * np.float32(h) >= 1.0
        rhs_ = -np.sum((w * h * h * kd * (Fp - kd * Yd) / (1 + kd * h))[asy])
        scale = np.sum(w * Yd) + h * np.sum(w * (Fp + kd * Yd))
        assert abs(np.sum(w * (Ynd - Yd)) - rhs_) <= 64 * F32_EPS * scale


@pytest.mark.parametrize("case", load_trace_cases(), ids=lambda c: c["name"])
def test_controller_hand_trace_in_float(case):
    """The hand-derived controller sequences hold in float: same accepted and rejected counts,
    the final state and step to float rounding."""
    k = case["k"]
    out = oracle.integrate_zone_f32(DECAY, np.array([k]), np.array([1.0, 1.0]), case["t_end"],
                                    case["dt0"])
    assert out["n_acc"] == case["n_acc"] and out["n_rej"] == case["n_rej"]
    ya = np.prod([(1.0 - k * h) ** n for h, acc, n in case["attempts"] if acc])
    assert out["Y"][0] == pytest.approx(ya, rel=2000 * F32_EPS)
    assert out["dt"] == pytest.approx(case["dt_out"], rel=1000 * F32_EPS)


def test_decay_converges_first_order_in_float():
    errs = []
    for tol in (1e-2, 1e-3):
        out = oracle.integrate_zone_f32(DECAY, np.array([10.0]), np.array([1.0, 0.0]), 1.0, 1e-6,
                                        oracle.options(tol=tol))
        assert out["status"] == oracle.ZONE_OK
        errs.append(abs(out["Y"][0] - math.exp(-10.0)) / math.exp(-10.0))
    assert errs[0] < 0.2 and 4.0 < errs[0] / errs[1] < 25.0


def test_euler_only_conserves_weight_to_float_rounding():
    wl = workloads.preset("n16_r48_const", n_zones=1)
    w = wl.network.weight.astype(np.float64)
    Y0 = wl.zones.Y0[0]
    out = oracle.integrate_zone_f32(wl.network, wl.zones.k[0], Y0, 1e-5, 1e-12,
                                    oracle.options(kappa=math.inf, max_steps=1000))
    assert out["n_acc"] > 20
    total0 = np.sum(w * Y0.astype(np.float32))
    assert abs(np.sum(w * out["Y"]) - total0) <= 2e-4 * total0


def test_float_and_double_agree_on_a_small_network():
    wl = workloads.preset("n16_r48_const", n_zones=4)
    a = oracle.integrate_batch(wl.network, wl.zones)
    b = oracle.integrate_batch(wl.network, wl.zones, precision=1)
    np.testing.assert_array_equal(b["status"], a["status"])
    assert np.all(np.abs(b["n_acc"] - a["n_acc"]) <= 0.01 * a["n_acc"])
    big = a["Y"] > 1e-6
    assert np.max(np.abs(b["Y"] - a["Y"])[big] / a["Y"][big]) < 1e-3


def test_statuses_in_float():
    ok = dict(k=np.array([1.0]), Y0=np.array([1.0, 0.0]), t_end=1.0, dt0=1e-3)
    for change, status in [(dict(k=np.array([np.nan])), oracle.ZONE_NONFINITE),
                           (dict(Y0=np.array([-1.0, 0.0])), oracle.ZONE_BAD_INPUT),
                           (dict(dt0=0.0), oracle.ZONE_BAD_INPUT),
                           (dict(t_end=0.0), oracle.ZONE_OK)]:
        args = dict(ok, **change)
        out = oracle.integrate_zone_f32(DECAY, args["k"], args["Y0"], args["t_end"], args["dt0"])
        assert out["status"] == status


@pytest.mark.parametrize("split_above,offset", [(0, 0), (8, 36), (12, 36), (39, 24), (40, 0)])
def test_long_rows_summed_in_chunks_in_float(split_above, offset):
    """The chunked row sums in float: 2^24 plus 39 ones.  One pass loses every +1 (ties to even);
    in chunks of c terms the row is 2^24 + (40 - c) exactly."""
    from tests.test_oracle_pins import long_row_net, long_row_sums

    net = long_row_net()
    fp, kd = long_row_sums(net, 2.0 ** 24, 1.0, split_above, rhs=oracle.rhs_f32, dtype=np.float32)
    assert fp == kd == np.float32(2.0 ** 24 + offset)
