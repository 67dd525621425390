"""GPU single-precision integration (asy_options.precision = ASY_PREC_F32) against the oracle's
single-precision integration on the same seeded zones.

Both sides evaluate the same float expressions in the same order (rates and abundances rounded
from double once per zone, the step-size rule in double), so constant-rate zones match bit for
bit.  Bar: relative error <= 1e-5 on every species whose oracle abundance exceeds 1e-30,
accepted steps within 1 % per zone, identical status; the tolerance covers Arrhenius zones whose
double rates (device vs host exp, last bit) round to different floats.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1409_5826_amd import binding, workloads

pytestmark = pytest.mark.gpu

REL_TOL = 1e-5
Y_MIN = 1e-30


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch

    assert torch.cuda.is_available(), "gpu tests need a device"
    binding.lib()
    yield


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def run_gpu(wl, zones=None, launch=None, precision=binding.PREC_F32, **opt):
    import torch

    zones = wl.zones if zones is None else zones
    net = binding.Network(wl.network)
    try:
        if launch:
            net.set_launch(**launch)
        buf = net.zone_buffers(zones)
        net.integrate(buf, binding.options_default(precision=precision, **opt))
        torch.cuda.synchronize()
        return {k: (None if v is None else v.cpu().numpy()) for k, v in buf.items()}
    finally:
        net.close()


def compare(g, ref, idx=None):
    sel = slice(None) if idx is None else np.asarray(idx)
    gY, gacc, gst = g["Y"][sel], g["n_accepted"][sel], g["zone_status"][sel]
    np.testing.assert_array_equal(gst, ref["status"])
    assert (np.abs(gacc - ref["n_acc"]) <= 0.01 * ref["n_acc"]).all()
    big = ref["Y"] > Y_MIN
    rel = np.abs(gY - ref["Y"])[big] / ref["Y"][big]
    assert rel.max(initial=0.0) <= REL_TOL, f"max rel err {rel.max():.3e}"
    return float(np.mean([np.array_equal(gY[i], ref["Y"][i]) for i in range(len(gY))]))


def test_n16_bit_exact():
    wl = workloads.preset("n16_r48_const", n_zones=8)
    say("case f32 n16_r48_const zones=8")
    g = run_gpu(wl)
    ref = oracle.integrate_batch(wl.network, wl.zones, precision=1)
    assert compare(g, ref) == 1.0
    np.testing.assert_array_equal(g["dt"], ref["dt"])


def test_n150_constant_rates_128_zones():
    wl = workloads.preset("n150_r1604_const")
    say("case f32 n150_r1604_const zones=128")
    g = run_gpu(wl)
    ref = oracle.integrate_batch(wl.network, wl.zones, precision=1)
    exact = compare(g, ref)
    say(f"  bit-exact zones {exact:.3f}")
    assert exact == 1.0


@pytest.mark.parametrize("name", ["n150_r1604_arrhenius", "n365_r4400_arrhenius"])
def test_arrhenius_full_size_every_zone(name):
    wl = workloads.preset(name)
    say(f"case f32 {name} zones={wl.zones.n_zones} all zones")
    g = run_gpu(wl)
    ref = oracle.integrate_batch(wl.network, wl.zones, precision=1)
    exact = compare(g, ref)
    say(f"  bit-exact zones {exact:.3f}")
    assert (g["zone_status"] == binding.ZONE_OK).all()
    for key, gkey in (("Y", "Y"), ("dt", "dt"), ("n_acc", "n_accepted"), ("n_rej", "n_rejected")):
        np.testing.assert_array_equal(g[gkey], ref[key], err_msg=key)


def test_placement_invariance_f32():
    wl = workloads.preset("n150_r1604_const", n_zones=24)
    say("case f32 placement n150_r1604_const zones=24")
    outs = [run_gpu(wl, launch=dict(variant=1, threads_per_zone=64 * W, zone_order=zo))
            for W, zo in [(1, 0), (2, 1), (4, 1)]]
    for o in outs[1:]:
        for key in ("Y", "dt", "n_accepted", "n_rejected", "zone_status"):
            np.testing.assert_array_equal(o[key], outs[0][key])


def test_f32_close_to_f64():
    wl = workloads.preset("n16_r48_const", n_zones=16)
    say("case f32 vs f64 n16_r48_const zones=16")
    g32 = run_gpu(wl)
    g64 = run_gpu(wl, precision=binding.PREC_F64)
    # a characterisation, not parity: float rounding of the state, worst over 16 zones
    big = g64["Y"] > 1e-6
    rel = np.abs(g32["Y"] - g64["Y"])[big] / g64["Y"][big]
    assert rel.max() < 1e-2 and np.median(rel) < 1e-4
    assert (np.abs(g32["n_accepted"] - g64["n_accepted"]) <= 0.01 * g64["n_accepted"]).all()


def test_f32_unsupported_combinations():
    import torch

    wl = workloads.preset("n16_r48_const", n_zones=2)
    net = binding.Network(wl.network)
    try:
        buf = net.zone_buffers(wl.zones)
        f32 = binding.options_default(precision=binding.PREC_F32)
        trace = torch.zeros((8, binding.TRACE_REC), dtype=torch.float32, device="cuda")
        count = torch.zeros(1, dtype=torch.int64, device="cuda")
        with pytest.raises(binding.AsyError) as e:
            net.integrate_trace(buf, trace, count, opts=f32)
        assert e.value.status == binding.ASY_ENOTSUP
        with pytest.raises(binding.AsyError) as e:
            net.integrate(buf, binding.options_default(precision=binding.PREC_F32,
                                                       controller=binding.CTRL_LEARNED))
        assert e.value.status == binding.ASY_ENOTSUP
        with pytest.raises(binding.AsyError) as e:
            net.integrate(buf, binding.options_default(precision=5))
        assert e.value.status == binding.ASY_EINVAL
        net.set_launch(variant=0, threads_per_zone=128, zone_order=0)
        with pytest.raises(binding.AsyError) as e:
            net.integrate(buf, f32)
        assert e.value.status == binding.ASY_ENOTSUP
        # the autotuner in single precision keeps to variant 1
        best = binding.asy_autotune(net.handle, net.n_species, net.n_reactions, buf["Y"],
                                    buf["t_end"], buf["dt"], k_zone=buf["k_zone"], opts=f32)
        assert best.variant == 1
        torch.cuda.synchronize()
    finally:
        net.close()
