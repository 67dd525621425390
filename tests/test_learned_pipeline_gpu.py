"""GPU: the trace -> training -> learned-integration pipeline of paper_1409_5826_amd.learned.

Checks the plumbing end to end on a small C2-distribution batch: trace records
carry finite features and boundary labels on the step grid (log2 0.9 + q/32);
the split keeps zones whole; training with the library's
kernels lowers the training loss on a learnable target; and the trained
network drives the learned controller to t_end in every zone.
"""
import sys

import numpy as np
import pytest

from paper_1409_5826_amd import binding, learned, workloads

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available()
    binding.lib()
    return torch


def small_batch(n_zones, t_scale, seed_offset):
    wl = workloads.preset("n150_r1604_const", n_zones=n_zones, seed_offset=seed_offset)
    z = wl.zones
    z.t_end = z.t_end * t_scale
    return wl, z


def test_traces_split_and_training(torch_dev):
    torch = torch_dev
    say("case learned pipeline: traces of 12 zones, split, training")
    wl, zones = small_batch(12, 0.05, 2003)
    net = binding.Network(wl.network)
    try:
        tr = learned.generate_traces(net, zones, 1e-2, stride=1, capacity=600000)
        assert tr.taken <= 600000 and len(tr.zone) > 1000
        assert bool(torch.isfinite(tr.x).all()) and bool(torch.isfinite(tr.y).all())
        # boundary labels: log2(0.9) + q/32 with q in [-96, 96], the largest accepted step of
        # the grid; the plain controller runs near r = 0.9 tol, so most labels sit near 0
        y = tr.y.cpu().numpy().astype(np.float64) - np.log2(0.9)
        assert y.max() <= 3.0 + 1e-5 and y.min() >= -3.0 - 1e-5
        np.testing.assert_allclose(32 * y, np.rint(32 * y), rtol=0, atol=1e-3)
        assert np.median(np.abs(y)) < 0.5
        sub = learned.subsample(tr, 8000, 7)
        assert len(sub.zone) == 8000 and np.all(np.diff(sub.n_acc[sub.zone == sub.zone[0]]) > 0)
        a, b = learned.split_by_zone(sub, 0.25, 7)
        assert len(a.zone) + len(b.zone) == 8000
        assert not set(np.unique(a.zone)) & set(np.unique(b.zone))
        # a learnable target on the recorded features: training must fit it
        target = (0.5 * a.x[:, 0] - 0.3 * a.x[:, wl.network.n_species + 2]).contiguous()
        target_v = (0.5 * b.x[:, 0] - 0.3 * b.x[:, wl.network.n_species + 2]).contiguous()
        fit_a = learned.Traces(x=a.x, y=target, zone=a.zone, n_acc=a.n_acc, taken=a.taken)
        fit_b = learned.Traces(x=b.x, y=target_v, zone=b.zone, n_acc=b.n_acc, taken=b.taken)
        res = learned.train(fit_a, fit_b, epochs=20, batch=512, lr=2e-3, seed=11)
        say(f"  train loss {res.train_loss[0]:.4g} -> {res.train_loss[-1]:.4g}, val "
            f"{res.val_loss[-1]:.4g} (mean predictor {res.baseline_val_loss:.4g})")
        assert res.train_loss[-1] < 0.25 * res.train_loss[0]
        assert res.val_loss[-1] < 0.5 * res.baseline_val_loss
        # the plain-trace labels themselves: training runs and stays finite
        res2 = learned.train(a, b, epochs=2, batch=512, lr=1e-3, seed=12)
        assert np.isfinite(res2.train_loss).all() and np.isfinite(res2.val_loss).all()
        # the trained network in the integrator (a briefly trained network may shrink the
        # step instead of keeping it, so the run is bounded by a step budget)
        net.set_mlp(res2.mlp)
        run = learned.integrate(net, zones, 1e-2, True, repeats=1, max_steps=100_000)
        assert np.isin(run.status, [binding.ZONE_OK, binding.ZONE_MAX_STEPS]).all()
        assert np.isfinite(run.Y).all() and (run.Y >= 0).all()
        plain = learned.integrate(net, zones, 1e-2, False, repeats=1)
        assert (plain.status == binding.ZONE_OK).all()
        say(f"  accepted steps learned {run.n_acc.sum()} plain {plain.n_acc.sum()}; rejected "
            f"learned {run.n_rej.sum()} plain {plain.n_rej.sum()}; learned statuses "
            f"{np.bincount(run.status, minlength=5)}")
        res.mlp.close()
        res2.mlp.close()
    finally:
        net.close()
