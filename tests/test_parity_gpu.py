"""GPU parity: the HIP integrator against the CPU oracle on the same seeded zones.

Bar: for every species whose oracle abundance exceeds 1e-20, relative error
<= 1e-9; accepted steps within 1% per zone; identical zone status; next-step
dt within 1e-9.  Both sides evaluate the same FP64 expressions in the same
order without contraction, so most zones agree bit for bit; the tolerance
absorbs the last-bit differences of exp() between the device and host math
libraries in the Arrhenius rates.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from paper_1409_5826_amd import binding, workloads

pytestmark = pytest.mark.gpu

REL_TOL = 1e-9
Y_MIN = 1e-20


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch

    assert torch.cuda.is_available(), "gpu tests need a device"
    binding.lib()
    yield


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def run_gpu(wl, opts=None, launch=None, zones=None):
    import torch

    zones = wl.zones if zones is None else zones
    net = binding.Network(wl.network)
    try:
        if launch:
            net.set_launch(**launch)
        buf = net.zone_buffers(zones)
        net.integrate(buf, opts)
        torch.cuda.synchronize()
        return {k: (None if v is None else v.cpu().numpy()) for k, v in buf.items()}
    finally:
        net.close()


def oracle_opts(o):
    if o is None:
        return oracle.options()
    return oracle.options(kappa=o.kappa, tol=o.tol, y_floor=o.y_floor, grow_max=o.grow_max,
                          safety=o.safety, shrink_min=o.shrink_min, dt_min=o.dt_min,
                          max_steps=o.max_steps)


def compare(g, ref, idx=None):
    """Assert parity of GPU outputs g (optionally rows idx) with oracle outputs ref."""
    sel = slice(None) if idx is None else np.asarray(idx)
    gY, gacc, grej = g["Y"][sel], g["n_accepted"][sel], g["n_rejected"][sel]
    gst, gdt = g["zone_status"][sel], g["dt"][sel]
    np.testing.assert_array_equal(gst, ref["status"])
    assert (np.abs(gacc - ref["n_acc"]) <= 0.01 * ref["n_acc"]).all()
    big = ref["Y"] > Y_MIN
    rel = np.abs(gY - ref["Y"])[big] / ref["Y"][big]
    assert rel.max(initial=0.0) <= REL_TOL, f"max rel err {rel.max():.3e}"
    np.testing.assert_allclose(gdt, ref["dt"], rtol=REL_TOL, atol=0)
    exact = np.mean([np.array_equal(gY[i], ref["Y"][i]) for i in range(len(gY))])
    return dict(max_rel=float(rel.max(initial=0.0)), bit_exact_zones=float(exact),
                steps=int(ref["n_acc"].sum()))


def test_n16_single_zone():
    wl = workloads.preset("n16_r48_const")
    say(f"case n16_r48_const zones={wl.zones.n_zones}")
    g = run_gpu(wl)
    ref = oracle.integrate_batch(wl.network, wl.zones)
    info = compare(g, ref)
    assert info["bit_exact_zones"] == 1.0   # constant rates: identical arithmetic
    assert g["n_accepted"][0] == ref["n_acc"][0] and g["n_rejected"][0] == ref["n_rej"][0]


def test_n150_constant_rates_128_zones():
    wl = workloads.preset("n150_r1604_const")
    say(f"case n150_r1604_const zones={wl.zones.n_zones}")
    g = run_gpu(wl)
    ref = oracle.integrate_batch(wl.network, wl.zones)
    info = compare(g, ref)
    assert info["bit_exact_zones"] == 1.0
    np.testing.assert_array_equal(g["n_accepted"], ref["n_acc"])
    np.testing.assert_array_equal(g["n_rejected"], ref["n_rej"])


@pytest.mark.parametrize("name", ["n150_r1604_arrhenius", "n365_r4400_arrhenius"])
def test_arrhenius_full_size_every_zone(name):
    """Full zone count in the default launch configuration; every zone against the oracle."""
    import time

    wl = workloads.preset(name)
    say(f"case {name} zones={wl.zones.n_zones} all zones")
    g = run_gpu(wl)
    t0 = time.perf_counter()
    ref = oracle.integrate_batch(wl.network, wl.zones)
    info = compare(g, ref)
    say(f"  oracle {time.perf_counter() - t0:.1f} s; max rel {info['max_rel']:.2e}, "
        f"bit-exact zones {info['bit_exact_zones']:.3f}, accepted steps equal in "
        f"{np.mean(g['n_accepted'] == ref['n_acc']):.4f} of zones")
    assert (g["zone_status"] == binding.ZONE_OK).all()
    assert (g["Y"] >= 0).all()
    # the rates' exponential is one algorithm on both sides, so every zone is identical
    for key, gkey in (("Y", "Y"), ("dt", "dt"), ("n_acc", "n_accepted"), ("n_rej", "n_rejected")):
        np.testing.assert_array_equal(g[gkey], ref[key], err_msg=key)


def test_arrhenius_small_batch_all_zones():
    wl = workloads.preset("n150_r1604_arrhenius", n_zones=67)   # ragged: not a multiple of anything
    say("case n150_r1604_arrhenius zones=67 all")
    g = run_gpu(wl)
    ref = oracle.integrate_batch(wl.network, wl.zones)
    compare(g, ref)


LAUNCHES = [
    dict(variant=0, threads_per_zone=64, zones_per_group=1, groups_per_cu=0, zone_order=0),
    dict(variant=0, threads_per_zone=128, zones_per_group=1, groups_per_cu=1, zone_order=0),
    dict(variant=0, threads_per_zone=512, zones_per_group=1, groups_per_cu=0, zone_order=0),
    dict(variant=1, threads_per_zone=64, zones_per_group=1, groups_per_cu=0, zone_order=1),
    dict(variant=1, threads_per_zone=128, zones_per_group=1, groups_per_cu=2, zone_order=0),
    dict(variant=1, threads_per_zone=256, zones_per_group=1, groups_per_cu=0, zone_order=1),
    dict(variant=1, threads_per_zone=128, zones_per_group=1, groups_per_cu=0, use_graph=1,
         zone_order=1),
]


@pytest.mark.parametrize("name", ["n150_r1604_const", "n150_r1604_arrhenius"])
def test_placement_invariance_and_determinism(name):
    """Kernel variant and launch configuration change only the speed: results are bit-identical."""
    wl = workloads.preset(name, n_zones=24)
    say(f"case placement {name} zones=24")
    outs = [run_gpu(wl, launch=c) for c in LAUNCHES]
    outs.append(run_gpu(wl, launch=LAUNCHES[3]))
    for o in outs[1:]:
        for key in ("Y", "dt", "n_accepted", "n_rejected", "zone_status"):
            np.testing.assert_array_equal(o[key], outs[0][key])


def test_graph_replay_repeats_and_autotune():
    """A captured graph replayed several times, with eager calls in between, matches eager runs;
    the autotuner returns a configuration that runs and gives the same results."""
    import torch

    wl = workloads.preset("n150_r1604_arrhenius", n_zones=40)
    say("case graph replay and autotune")
    eager = run_gpu(wl)
    net = binding.Network(wl.network)
    try:
        net.set_launch(use_graph=1)
        buf = net.zone_buffers(wl.zones)
        Y0, dt0 = buf["Y"].clone(), buf["dt"].clone()
        for rep in range(3):
            buf["Y"].copy_(Y0)
            buf["dt"].copy_(dt0)
            net.integrate(buf)
            torch.cuda.synchronize()
            for key in ("Y", "dt", "n_accepted", "n_rejected", "zone_status"):
                np.testing.assert_array_equal(buf[key].cpu().numpy(), eager[key])
            z = torch.zeros(1000, device="cuda").sum()   # eager work between replays
            torch.cuda.synchronize()
            assert float(z) == 0.0
        best = binding.asy_autotune(net.handle, net.n_species, net.n_reactions, Y0, buf["t_end"], dt0,
                                    T=buf["T"], sample_zones=40)
        say(f"autotuned: {best.as_dict()}")
        assert net.get_launch() == best.as_dict()
        buf["Y"].copy_(Y0)
        buf["dt"].copy_(dt0)
        net.integrate(buf)
        torch.cuda.synchronize()
        for key in ("Y", "dt", "n_accepted", "n_rejected", "zone_status"):
            np.testing.assert_array_equal(buf[key].cpu().numpy(), eager[key])
    finally:
        net.close()


def test_edge_cases_statuses():
    """Bad inputs, budgets and degenerate intervals, zone by zone, against the oracle."""
    wl = workloads.preset("n150_r1604_const", n_zones=8)
    z = wl.zones
    z.Y0[1, 7] = np.nan          # non-finite abundance
    z.Y0[2, 3] = -1e-3           # negative abundance
    z.k[3, 11] = np.inf          # non-finite rate
    z.t_end[4] = 0.0             # empty interval
    z.dt0[5] = 0.0               # invalid trial step
    z.t_end[6] = 1e-9            # interval shorter than a few steps
    z.dt0[7] = 10.0              # trial step larger than the interval (clipped first step)
    say("case edge statuses")
    g = run_gpu(wl)
    ref = oracle.integrate_batch(wl.network, z)
    assert list(ref["status"][:6]) == [0, 3, 4, 3, 0, 4]
    compare(g, ref)
    np.testing.assert_array_equal(g["Y"][1:4], z.Y0[1:4])  # untouched on input failure


@pytest.mark.parametrize("kw,status", [(dict(max_steps=50), binding.ZONE_MAX_STEPS),
                                       (dict(dt_min=1e-6), binding.ZONE_DT_UNDERFLOW)])
def test_budget_statuses(kw, status):
    wl = workloads.preset("n150_r1604_const", n_zones=4)
    opts = binding.options_default(**kw)
    say(f"case budget {kw}")
    g = run_gpu(wl, opts=opts)
    ref = oracle.integrate_batch(wl.network, wl.zones, oracle_opts(opts))
    assert (ref["status"] == status).all()
    compare(g, ref)


def test_euler_only_and_tight_tolerance():
    wl = workloads.preset("n16_r48_const")
    for kw in (dict(kappa=math.inf, max_steps=2000), dict(tol=1e-4)):
        opts = binding.options_default(**kw)
        say(f"case n16 options {kw}")
        g = run_gpu(wl, opts=opts)
        ref = oracle.integrate_batch(wl.network, wl.zones, oracle_opts(opts))
        compare(g, ref)


def test_zero_zones_is_a_no_op():
    import torch

    wl = workloads.preset("n16_r48_const")
    net = binding.Network(wl.network)
    try:
        e = torch.empty((0, 16), dtype=torch.float64, device="cuda")
        z = torch.empty(0, dtype=torch.float64, device="cuda")
        i64 = torch.empty(0, dtype=torch.int64, device="cuda")
        i32 = torch.empty(0, dtype=torch.int32, device="cuda")
        kz = torch.empty((0, 48), dtype=torch.float64, device="cuda")
        binding.asy_integrate_batch(net.handle, 16, 48, e, z, z, i64, i64, i32, k_zone=kz)
        torch.cuda.synchronize()
    finally:
        net.close()


def test_layout_info_one_factor_waves_and_placement():
    # the packing frees whole waves of second gathers and the placement lowers the modelled
    # gather cycles; the integrations above run through these layouts
    cases = [("n150_r1604_arrhenius", 128, 0b10, 0, 32), ("n365_r4400_arrhenius", 256, 0b1100, 16, 56)]
    for name, tpz, waves, f1, c2 in cases:
        net = binding.Network(workloads.preset(name, n_zones=1).network)
        try:
            info = net.layout_info(tpz)
            say(f"layout {name} {tpz}: {info}")
            assert info["available"] == 1 and info["slots_used"] <= info["slots"]
            assert info["one_factor_waves"] == waves
            assert info["gather_cycles_placed"] < info["gather_cycles_packed"]
            # the two-factor rows sit in each lane's last slots; the leading ones run one-factor
            assert info["one_factor_slots"] >= f1 and info["one_factor_slots_run"] == f1
            # balanced layout (150 species): the two-factor wave stops at slot 32 of 44
            assert info["two_factor_wave_slots"] == c2
            with pytest.raises(binding.AsyError):
                net.layout_info(96)
        finally:
            net.close()


@pytest.mark.parametrize("tpz", [64, 128])
def test_one_body_network_every_wave_one_factor(tpz):
    # only one-body reactions: every second factor is the 1.0 cell, so every wave takes the
    # slot phase without second gathers; constant rates, bit for bit with the oracle
    net = workloads.make_network(72, 200, 0, mass_group=8, seed=7701)
    zones = workloads.make_zones(net, 12, seed=7702, t_end=1e-2, log10_k_range=(-4.0, 6.0))
    wl = workloads.Workload("one_body_n72", net, zones, 0.01, "one-body only")
    say(f"case one-body n72 zones=12 threads_per_zone={tpz}")
    h = binding.Network(net)
    try:
        info = h.layout_info(tpz)
    finally:
        h.close()
    assert info["one_factor_waves"] == (1 << (tpz // 64)) - 1
    g = run_gpu(wl, launch=dict(variant=1, threads_per_zone=tpz, zone_order=1))
    ref = oracle.integrate_batch(net, zones)
    assert compare(g, ref)["bit_exact_zones"] == 1.0
    np.testing.assert_array_equal(g["n_accepted"], ref["n_acc"])
