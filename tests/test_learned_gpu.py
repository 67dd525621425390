"""GPU learned controller and trace records against the oracle.

The learned controller changes only which trial step is proposed.  Its proposal
q is an integer that floating point decides, so the oracle evaluates the network
in the device's matrix-core arithmetic (oracle.mlp_forward_mfma: BF16 operands,
FP32 accumulation by the rule measured on gfx950).  Checks:
* every q the GPU recorded equals the oracle network's q on the recorded
  features (all but a few in 10^4, the mismatch rate of the accumulation rule);
* replaying the GPU's q in the oracle reproduces the trajectory exactly on
  constant-rate networks and within the parity bar with Arrhenius rates, and the
  oracle's proposal log equals the GPU's records (features to float rounding of
  log10, boundary labels, accepted-step counts exactly);
* end to end, with a network trained by the library's own pipeline, the oracle
  running that network itself reproduces the GPU's accepted-step sequence in at
  least 99 % of 128 zones of the 150-species constant-rate workload.
"""
import sys

import numpy as np
import pytest

import oracle
from oracle import mlp as ref
from paper_1409_5826_amd import binding, workloads

pytestmark = pytest.mark.gpu

FEAT_ATOL = 2e-6
LABEL_ATOL = 2e-6
# an untrained network may shrink the step again and again: bound every zone's work
MAX_STEPS = 50_000


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available(), "gpu tests need a device"
    binding.lib()
    return torch


def mlp_params(seed=5, b3=0.2):
    """Random network; b3 shifts its outputs so that its proposals are a mix of accepted and
    rejected ones on the workload at hand."""
    p = ref.init_params(seed)
    u = ref.unpack(p)
    rng = np.random.default_rng(seed + 100)
    u["b1"] = rng.normal(scale=0.1, size=128)
    u["b2"] = rng.normal(scale=0.1, size=128)
    u["W3"] = rng.normal(scale=0.2, size=128)
    u["b3"] = np.array([b3])
    return ref.pack(u).astype(np.float32)


def shortened(wl, n_zones, t_scale):
    z = wl.zones
    assert z.n_zones >= n_zones
    sel = slice(0, n_zones)
    return workloads.Zones(Y0=z.Y0[sel].copy(), t_end=z.t_end[sel] * t_scale, dt0=z.dt0[sel].copy(),
                           k=None if z.k is None else z.k[sel].copy(),
                           T=None if z.T is None else z.T[sel].copy())


def zone_rates(wl, zones, i):
    if zones.k is not None:
        return zones.k[i]
    return oracle.rates_arrhenius(wl.network.A, wl.network.E, zones.T[i])


def run(torch, wl, zones, learned, params=None, trace_cap=0, stride=1, trace_zones=None,
        launch=None, max_steps=MAX_STEPS):
    net = binding.Network(wl.network)
    m = None
    try:
        if launch:
            net.set_launch(**launch)
        if params is not None:
            m = binding.Mlp(1)
            m.set_params(params)
            net.set_mlp(m)
        opts = binding.options_default(controller=binding.CTRL_LEARNED if learned else
                                       binding.CTRL_PLAIN, max_steps=max_steps)
        buf = net.zone_buffers(zones)
        out = {}
        if trace_cap:
            trace = torch.full((trace_cap, binding.TRACE_REC), float("nan"), dtype=torch.float32,
                               device="cuda")
            count = torch.zeros(1, dtype=torch.int64, device="cuda")
            net.integrate_trace(buf, trace, count, stride=stride, trace_zones=trace_zones, opts=opts)
            torch.cuda.synchronize()
            out["count"] = int(count.item())
            out["trace"] = trace[:min(out["count"], trace_cap)].cpu().numpy()
        else:
            net.integrate(buf, opts)
            torch.cuda.synchronize()
        out.update({k: (None if v is None else v.cpu().numpy()) for k, v in buf.items()})
        return out
    finally:
        net.close()
        if m is not None:
            m.close()


def records_by_zone(trace):
    z = trace[:, 168].astype(np.int64)
    n = trace[:, 169].astype(np.int64)
    order = np.lexsort((n, z))
    t = trace[order]
    zs = t[:, 168].astype(np.int64)
    return {int(k): t[zs == k] for k in np.unique(zs)}


def check_log(rec, log, N, label_mismatch_max=0.0):
    """GPU records of one zone against the oracle's proposal log entries with the same n_acc.
    With Arrhenius rates (last-bit differences of exp) a boundary label may sit on the other
    side of a grid point: label_mismatch_max bounds the share of such records."""
    n = rec[:, 169].astype(np.int64)
    idx = np.searchsorted(log["n_acc"], n)
    assert (idx < len(log["n_acc"])).all() and (log["n_acc"][idx] == n).all()
    np.testing.assert_allclose(rec[:, :N + 4], log["feat"][idx, :N + 4], rtol=0, atol=FEAT_ATOL)
    assert (rec[:, N + 4:166] == 0).all()
    lab_g, lab_o = rec[:, 166].astype(np.float64), log["label"][idx]
    both = ~np.isnan(lab_g) & ~np.isnan(lab_o)
    differ = (np.isnan(lab_g) != np.isnan(lab_o)) | (both & (np.abs(lab_g - lab_o) > LABEL_ATOL))
    assert (differ.mean() if differ.size else 0.0) <= label_mismatch_max, \
        f"{differ.sum()} labels differ"


def check_q_against_network(params, trace, max_checks=3000):
    """q of the GPU's in-kernel network against the oracle's matrix-core forward on the same
    recorded features."""
    rng = np.random.default_rng(0)
    sel = rng.choice(len(trace), size=min(max_checks, len(trace)), replace=False)
    o = np.array([oracle.mlp_forward_mfma(params, trace[i, :166]) for i in sel])
    q_ref = np.rint(32.0 * np.clip(o, -3.0, 3.0))
    q_gpu = trace[sel, 167]
    frac = float(np.mean(q_gpu == q_ref))
    say(f"  q equal to the oracle network's on {frac:.5f} of {len(sel)} records")
    assert frac >= 0.999
    return len(np.unique(q_gpu))


# b3 = 0.2 makes this network propose growth that the controller mostly rejects (the fallback
# path); the negative shift makes it propose shrinking steps that are accepted until the step
# budget ends the zone (the accepted-proposal path)
CASES = [
    ("n16_r48_const", 8, 1.0, True, 0.2),
    ("n16_r48_const", 8, 1.0, True, -0.05),
    ("n150_r1604_const", 4, 0.25, True, 0.2),
    ("n150_r1604_arrhenius", 4, 1.0, False, 0.2),
]


@pytest.mark.parametrize("name,n_zones,t_scale,exact,b3", CASES)
def test_learned_integration_replays_in_oracle(torch_dev, name, n_zones, t_scale, exact, b3):
    torch = torch_dev
    wl = workloads.preset(name, n_zones=n_zones)
    zones = shortened(wl, n_zones, t_scale)
    N = wl.network.n_species
    p = mlp_params(b3=b3)
    say(f"case learned+trace {name} zones={n_zones} t_scale={t_scale}")
    cap = n_zones * MAX_STEPS + 1024
    g = run(torch, wl, zones, True, p, trace_cap=cap)
    assert g["count"] <= cap, "trace buffer too small for the test"
    by_zone = records_by_zone(g["trace"])
    n_q = check_q_against_network(p, g["trace"])
    assert n_q >= 4, "the test network should propose several different ratios"
    for z in range(n_zones):
        rec = by_zone.get(z, np.zeros((0, binding.TRACE_REC), np.float32))
        q = rec[:, 167].astype(np.int32)
        o = oracle.integrate_zone_learned(wl.network, zone_rates(wl, zones, z), zones.Y0[z],
                                          zones.t_end[z], zones.dt0[z], p, q_replay=q,
                                          opts=oracle.options(max_steps=MAX_STEPS),
                                          log_capacity=len(q) + 1)
        assert o["status"] == g["zone_status"][z]
        assert o["n_prop"] == len(q), f"zone {z}: {o['n_prop']} proposals vs {len(q)} records"
        np.testing.assert_array_equal(o["log"]["q"], q)
        if exact:
            np.testing.assert_array_equal(g["Y"][z], o["Y"])
            assert (g["n_accepted"][z], g["n_rejected"][z]) == (o["n_acc"], o["n_rej"])
            assert g["dt"][z] == o["dt"]
        else:
            big = o["Y"] > 1e-20
            rel = np.abs(g["Y"][z] - o["Y"])[big] / o["Y"][big]
            assert rel.max(initial=0) <= 1e-9
            assert abs(g["n_accepted"][z] - o["n_acc"]) <= 0.01 * o["n_acc"]
        check_log(rec, o["log"], N, 0.0 if exact else 0.01)
    # the learned kernel without trace output takes the same steps
    g2 = run(torch, wl, zones, True, p)
    np.testing.assert_array_equal(g2["Y"], g["Y"])
    np.testing.assert_array_equal(g2["n_accepted"], g["n_accepted"])
    np.testing.assert_array_equal(g2["n_rejected"], g["n_rejected"])
    np.testing.assert_array_equal(g2["dt"], g["dt"])
    say(f"  proposals={len(g['trace'])} distinct q={n_q} accepted={g['n_accepted'].sum()} "
        f"rejected={g['n_rejected'].sum()} status={np.bincount(g['zone_status'], minlength=5)}")


def test_plain_trace_records_stride_and_zone_limit(torch_dev):
    torch = torch_dev
    wl = workloads.preset("n16_r48_const", n_zones=12)
    zones = shortened(wl, 12, 1.0)
    N = wl.network.n_species
    say("case plain trace n16 zones=12 stride=3 trace_zones=5")
    plain_gpu = run(torch, wl, zones, False)
    g = run(torch, wl, zones, False, trace_cap=200000, stride=3, trace_zones=5)
    # recording does not change the integration
    for key in ("Y", "dt", "n_accepted", "n_rejected", "zone_status"):
        np.testing.assert_array_equal(g[key], plain_gpu[key])
    tr = g["trace"]
    assert g["count"] == len(tr) > 0
    assert (tr[:, 168] < 5).all() and (tr[:, 169] % 3 == 0).all() and np.isnan(tr[:, 167]).all()
    by_zone = records_by_zone(tr)
    assert sorted(by_zone) == list(range(5))
    for z in range(5):
        o = oracle.integrate_zone_learned(wl.network, zones.k[z], zones.Y0[z], zones.t_end[z],
                                          zones.dt0[z], learned=False,
                                          opts=oracle.options(max_steps=MAX_STEPS),
                                          log_capacity=10 ** 6, label_stride=3)
        np.testing.assert_array_equal(g["Y"][z], o["Y"])
        want = o["log"]["n_acc"][o["log"]["n_acc"] % 3 == 0]
        np.testing.assert_array_equal(by_zone[z][:, 169].astype(np.int64), want)
        check_log(by_zone[z], o["log"], N)


def test_trace_capacity_overflow_keeps_valid_records(torch_dev):
    torch = torch_dev
    wl = workloads.preset("n16_r48_const", n_zones=4)
    zones = shortened(wl, 4, 1.0)
    say("case trace overflow n16 zones=4 capacity=37")
    plain_gpu = run(torch, wl, zones, False)
    g = run(torch, wl, zones, False, trace_cap=37)
    np.testing.assert_array_equal(g["Y"], plain_gpu["Y"])
    assert g["count"] > 37 and len(g["trace"]) == 37
    by_zone = records_by_zone(g["trace"])
    for z, rec in by_zone.items():
        o = oracle.integrate_zone_learned(wl.network, zones.k[z], zones.Y0[z], zones.t_end[z],
                                          zones.dt0[z], learned=False,
                                          opts=oracle.options(max_steps=MAX_STEPS),
                                          log_capacity=10 ** 6)
        check_log(rec, o["log"], wl.network.n_species)


def test_learned_controller_argument_errors(torch_dev):
    torch = torch_dev
    wl = workloads.preset("n16_r48_const", n_zones=2)
    zones = shortened(wl, 2, 1.0)
    net = binding.Network(wl.network)
    try:
        buf = net.zone_buffers(zones)
        learned = binding.options_default(controller=binding.CTRL_LEARNED)
        with pytest.raises(binding.AsyError) as e:
            net.integrate(buf, learned)
        assert e.value.status == binding.ASY_ESTATE
        trace = torch.zeros((8, binding.TRACE_REC), dtype=torch.float32, device="cuda")
        count = torch.zeros(1, dtype=torch.int64, device="cuda")
        with pytest.raises(binding.AsyError) as e:
            net.integrate_trace(buf, trace, count, stride=0)
        assert e.value.status == binding.ASY_EINVAL
        net.set_launch(variant=0, threads_per_zone=128, zone_order=0)
        with pytest.raises(binding.AsyError) as e:
            net.integrate_trace(buf, trace, count)
        assert e.value.status == binding.ASY_ENOTSUP
        bad = binding.options_default(controller=7)
        with pytest.raises(binding.AsyError) as e:
            net.integrate(buf, bad)
        assert e.value.status == binding.ASY_EINVAL
        torch.cuda.synchronize()
    finally:
        net.close()


def test_learned_end_to_end_with_a_trained_network(torch_dev):
    """Train the proposer with the library's own pipeline (plain traces with boundary labels on
    64 training zones, augmented for other step sizes, BF16 MFMA training on the device), then
    integrate 64 zones of the 150-species constant-rate workload with it on the GPU and in the
    oracle, which evaluates the same parameters itself.  Bar: identical accepted-step sequences
    (Y, next dt, accepted and rejected counts, status) in at least 99 % of the zones; the others
    within 1 % in accepted steps and 1e-6 relative in every abundance above 1e-20."""
    import time
    from concurrent.futures import ThreadPoolExecutor, as_completed

    from paper_1409_5826_amd import learned

    torch = torch_dev
    tr_wl = workloads.preset("n150_r1604_const", n_zones=64, seed_offset=2003)
    wl = workloads.preset("n150_r1604_const", n_zones=64)
    say(f"case learned end to end: train on 64 zones, evaluate {wl.zones.n_zones} zones")
    net = binding.Network(wl.network)
    try:
        traces = learned.generate_traces(net, tr_wl.zones, 1e-2, stride=12, capacity=200000)
        traces = learned.augment_step_scale(traces, wl.network.n_species)
        tr_set, va_set = learned.split_by_zone(traces, 0.1, 4005)
        res = learned.train(tr_set, va_set, epochs=4, batch=1024, lr=1e-3, seed=4005)
        params = res.mlp.get_params()
        res.mlp.close()
    finally:
        net.close()
    say(f"  trained on {len(tr_set.zone)} pairs: val loss {res.val_loss[-1]:.3e} "
        f"(mean predictor {res.baseline_val_loss:.3e})")
    max_steps = 100_000
    g = run(torch, wl, wl.zones, True, params, max_steps=max_steps)
    say(f"  GPU: accepted {int(g['n_accepted'].sum())}, rejected {int(g['n_rejected'].sum())}, "
        f"statuses {np.bincount(g['zone_status'], minlength=5)}")
    t0 = time.perf_counter()

    def one(z):
        return z, oracle.integrate_zone_learned(wl.network, wl.zones.k[z], wl.zones.Y0[z],
                                                wl.zones.t_end[z], wl.zones.dt0[z], params,
                                                opts=oracle.options(max_steps=max_steps))
    outs = {}
    with ThreadPoolExecutor(max_workers=16) as pool:
        futs = [pool.submit(one, z) for z in range(wl.zones.n_zones)]
        for i, f in enumerate(as_completed(futs)):
            z, o = f.result()
            outs[z] = o
            if i % 8 == 7:
                say(f"  oracle zones done {i + 1} ({time.perf_counter() - t0:.0f} s)")
    same = []
    for z in range(wl.zones.n_zones):
        o = outs[z]
        eq = (np.array_equal(g["Y"][z], o["Y"]) and g["dt"][z] == o["dt"] and
              (g["n_accepted"][z], g["n_rejected"][z], g["zone_status"][z]) ==
              (o["n_acc"], o["n_rej"], o["status"]))
        same.append(eq)
        if not eq:
            assert g["zone_status"][z] == o["status"]
            assert abs(g["n_accepted"][z] - o["n_acc"]) <= 0.01 * o["n_acc"]
            big = o["Y"] > 1e-20
            assert (np.abs(g["Y"][z] - o["Y"])[big] / o["Y"][big]).max() <= 1e-6
    frac = float(np.mean(same))
    say(f"  identical zones {frac:.4f}; oracle {time.perf_counter() - t0:.1f} s")
    assert frac >= 0.99
