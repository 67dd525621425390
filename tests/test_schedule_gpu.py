"""GPU operator-split schedule (asy_integrate_schedule) against the oracle's schedule: abundances,
carried trial steps, summed counters, first-failure statuses and the energy released per step."""
import sys

import numpy as np
import pytest

import oracle
from paper_1409_5826_amd import binding, workloads

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch

    assert torch.cuda.is_available()
    binding.lib()
    yield


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def run(wl, sched, precision=0, **opt):
    import torch

    net = binding.Network(wl.network)
    try:
        buf = net.zone_buffers(wl.zones)
        energy = net.integrate_schedule(buf, sched, binding.options_default(precision=precision,
                                                                            **opt))
        torch.cuda.synchronize()
        out = {k: (None if v is None else v.cpu().numpy()) for k, v in buf.items()}
        out["energy"] = energy.cpu().numpy()
        return out
    finally:
        net.close()


def test_constant_rates_bit_exact():
    wl = workloads.preset("n150_r1604_const", n_zones=16)
    sched = workloads.make_schedule(wl.network, wl.zones, 5, seed=11)
    say("case schedule n150_r1604_const zones=16 steps=5")
    g = run(wl, sched)
    ref = oracle.integrate_schedule(wl.network, wl.zones, sched)
    for key, gkey in (("Y", "Y"), ("dt", "dt"), ("n_acc", "n_accepted"), ("n_rej", "n_rejected"),
                      ("status", "zone_status"), ("energy", "energy")):
        np.testing.assert_array_equal(g[gkey], ref[key])


@pytest.mark.parametrize("precision", [0, 1])
def test_arrhenius_temperature_path_bit_exact(precision):
    """Arrhenius rates along a temperature path: both sides evaluate the rates' exponential by the
    same algorithm, so the schedule matches the oracle's bit for bit, energies included, in
    double and in single precision."""
    wl = workloads.preset("n150_r1604_arrhenius", n_zones=256)
    sched = workloads.make_schedule(wl.network, wl.zones, 4, seed=12, T_swing=0.2)
    say(f"case schedule n150_r1604_arrhenius zones=256 steps=4 precision={precision}")
    g = run(wl, sched, precision=precision)
    ref = oracle.integrate_schedule(wl.network, wl.zones, sched, precision=precision)
    for key, gkey in (("Y", "Y"), ("dt", "dt"), ("n_acc", "n_accepted"), ("n_rej", "n_rejected"),
                      ("status", "zone_status"), ("energy", "energy")):
        np.testing.assert_array_equal(g[gkey], ref[key], err_msg=key)


def test_schedule_argument_errors():
    import torch

    wl = workloads.preset("n16_r48_const", n_zones=2)
    net = binding.Network(wl.network)
    try:
        buf = net.zone_buffers(wl.zones)
        dt_h = torch.full((3, 2), 1e-3, dtype=torch.float64, device="cuda")
        energy = torch.zeros((3, 2), dtype=torch.float64, device="cuda")
        with pytest.raises(binding.AsyError) as e:
            binding.asy_integrate_schedule(net.handle, net.n_species, net.n_reactions, buf["Y"],
                                           dt_h, buf["dt"], buf["n_accepted"], buf["n_rejected"],
                                           buf["zone_status"], k_zone=buf["k_zone"], energy=energy)
        assert e.value.status == binding.ASY_EINVAL
        empty = torch.zeros((0, 2), dtype=torch.float64, device="cuda")
        with pytest.raises(binding.AsyError) as e:
            binding.asy_integrate_schedule(net.handle, net.n_species, net.n_reactions, buf["Y"],
                                           empty, buf["dt"], buf["n_accepted"], buf["n_rejected"],
                                           buf["zone_status"], k_zone=buf["k_zone"])
        assert e.value.status == binding.ASY_EINVAL
        torch.cuda.synchronize()
    finally:
        net.close()
