"""GPU integration of a network with hub species (3 species in about 200 reactions each).

Rows of more than 64 terms are summed in chunks of 32 consecutive terms whose partial sums are
then added in order.  The oracle sums rows in that order too when asked (options split_above),
so the GPU must match it bit for bit, in double and in single precision; against the oracle's
one-pass sums the chunked order moves results by a few ulps per sum, which the stiff steps carry
to at most 1e-8 relative.  The chunking does not depend on the launch, so all launch
configurations agree bit for bit.
"""
import sys

import numpy as np
import pytest

import oracle
from paper_1409_5826_amd import binding, workloads

pytestmark = pytest.mark.gpu

NAME = "n150_r1604_hub_arrhenius"


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch

    assert torch.cuda.is_available()
    binding.lib()
    yield


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def run(wl, launch=None, precision=0):
    import torch

    net = binding.Network(wl.network)
    try:
        if launch:
            net.set_launch(**launch)
        used = net.get_launch()
        buf = net.zone_buffers(wl.zones)
        net.integrate(buf, binding.options_default(precision=precision))
        torch.cuda.synchronize()
        out = {k: (None if v is None else v.cpu().numpy()) for k, v in buf.items()}
        out["launch"] = used
        return out
    finally:
        net.close()


def check(g, ref, idx, rel_tol, y_min):
    np.testing.assert_array_equal(g["zone_status"][idx], ref["status"])
    assert (np.abs(g["n_accepted"][idx] - ref["n_acc"]) <= 0.01 * ref["n_acc"]).all()
    big = ref["Y"] > y_min
    rel = np.abs(g["Y"][idx] - ref["Y"])[big] / ref["Y"][big]
    assert rel.max() <= rel_tol, f"max rel {rel.max():.3e}"
    return rel.max()


def test_hub_network_is_split_and_packed():
    wl = workloads.preset(NAME, n_zones=4)
    net = wl.network
    kd = np.bincount(net.reactant0, minlength=150) + np.bincount(net.reactant1[net.reactant1 >= 0],
                                                                 minlength=150)
    assert np.sort(kd)[-3:].min() > 150  # three hub rows of ~200 terms
    h = binding.Network(net)
    try:
        launch = h.get_launch()
        # default launch: the packed kernel, not the generic fallback
        assert launch["variant"] == 1 and launch["threads_per_zone"] == 128
    finally:
        h.close()


def same(g, ref, idx=None):
    idx = slice(None) if idx is None else idx
    np.testing.assert_array_equal(g["zone_status"][idx], ref["status"])
    np.testing.assert_array_equal(g["n_accepted"][idx], ref["n_acc"])
    np.testing.assert_array_equal(g["n_rejected"][idx], ref["n_rej"])
    np.testing.assert_array_equal(g["dt"][idx], ref["dt"])
    np.testing.assert_array_equal(g["Y"][idx], ref["Y"])


def test_hub_parity_full_batch_every_zone():
    """Every zone of the hub batch, bit for bit against the oracle summing long rows in the same
    chunks.  Against the one-pass oracle (definition order) each hub sum differs by a few ulps,
    which a few species that come out of a near-cancellation carry further over thousands of
    stiff steps: statuses equal, accepted steps within 1 %, every species above 1e-20 within
    1e-8 relative and all but 1 in 1e5 within 1e-9."""
    wl = workloads.preset(NAME)
    say(f"case hub {NAME} zones={wl.zones.n_zones} all zones")
    g = run(wl)
    same(g, oracle.integrate_batch(wl.network, wl.zones, opts=oracle.options(split_above=64)))
    ref = oracle.integrate_batch(wl.network, wl.zones)
    np.testing.assert_array_equal(g["zone_status"], ref["status"])
    assert (np.abs(g["n_accepted"] - ref["n_acc"]) <= 0.01 * ref["n_acc"]).all()
    big = ref["Y"] > 1e-20
    rel = np.abs(g["Y"] - ref["Y"])[big] / ref["Y"][big]
    over = float(np.mean(rel > 1e-9))
    say(f"  bit-exact against the chunked oracle; against one pass: max rel {rel.max():.2e}, "
        f"median {np.median(rel):.1e}, share above 1e-9 {over:.1e}; launch {g['launch']}")
    assert rel.max() <= 1e-8 and over <= 1e-5
    assert (g["zone_status"] == binding.ZONE_OK).all()


def test_hub_launch_invariance():
    wl = workloads.preset(NAME, n_zones=48)
    say("case hub launch invariance zones=48")
    outs = [run(wl, launch=dict(variant=1, threads_per_zone=64 * W, zone_order=zo))
            for W, zo in [(1, 1), (2, 1), (4, 0)]]
    for o in outs[1:]:
        for key in ("Y", "dt", "n_accepted", "n_rejected", "zone_status"):
            np.testing.assert_array_equal(o[key], outs[0][key])


def test_hub_f32_full_batch_every_zone():
    """Single precision, every zone of the hub batch, bit for bit against the single-precision
    oracle summing long rows in the same chunks."""
    wl = workloads.preset(NAME)
    say(f"case hub f32 {NAME} zones={wl.zones.n_zones} all zones")
    g32 = run(wl, precision=1)
    same(g32, oracle.integrate_batch(wl.network, wl.zones, opts=oracle.options(split_above=64),
                                     precision=1))


def test_split_threshold_option():
    """A lower split threshold (split_above) chunks the ordinary rows too: the results match the
    oracle summing in the same chunks bit for bit, stay within the parity bar of the one-pass
    oracle and do not depend on the launch."""
    import torch

    wl = workloads.preset("n150_r1604_arrhenius", n_zones=24)
    say("case split_above=24 n150_r1604_arrhenius zones=24")
    outs = []
    for W in (2, 4):
        net = binding.Network(wl.network, split_above=24)
        try:
            net.set_launch(variant=1, threads_per_zone=64 * W, zone_order=1)
            buf = net.zone_buffers(wl.zones)
            net.integrate(buf)
            torch.cuda.synchronize()
            outs.append({k: (None if v is None else v.cpu().numpy()) for k, v in buf.items()})
        finally:
            net.close()
    for key in ("Y", "dt", "n_accepted", "n_rejected", "zone_status"):
        np.testing.assert_array_equal(outs[1][key], outs[0][key])
    same(outs[0], oracle.integrate_batch(wl.network, wl.zones,
                                         opts=oracle.options(split_above=24)))
    ref = oracle.integrate_batch(wl.network, wl.zones)
    say(f"  bit-exact against the oracle in chunks of 12; against one pass max rel "
        f"{check(outs[0], ref, np.arange(24), 1e-9, 1e-20):.2e}")
