"""The entry point that allocates nothing (asy_integrate_batch_noalloc) against
asy_integrate_batch, through the C ABI: identical outputs, bit for bit, on two
calls in a row, the second with fewer zones (the static scratch keeps the first
call's keys and order; the second must not see them)."""
import ctypes as C
import sys

import numpy as np
import pytest

from paper_1409_5826_amd import binding, workloads

pytestmark = pytest.mark.gpu

FIELDS = ("Y", "dt", "n_accepted", "n_rejected", "zone_status")


@pytest.fixture(scope="module", autouse=True)
def _device():
    import torch

    assert torch.cuda.is_available(), "gpu tests need a device"
    binding.lib()
    yield


def say(msg):
    print(msg, file=sys.stderr, flush=True)


def _run(net, zones, noalloc, opts=None):
    import torch

    buf = net.zone_buffers(zones)
    net.integrate(buf, opts, noalloc=noalloc)
    torch.cuda.synchronize()
    return {k: buf[k].cpu().numpy() for k in FIELDS}


def _same(a, b):
    for k in FIELDS:
        np.testing.assert_array_equal(a[k], b[k], err_msg=k)


@pytest.mark.parametrize("name,n1,n2,launch", [
    ("n150_r1604_arrhenius", 300, 67, None),                       # longest-first order
    ("n150_r1604_arrhenius", 200, 33, {"zone_order": 0}),          # index order
    ("n150_r1604_const", 128, 40, None),                           # per-zone rates
    ("n16_r48_const", 1, 1, {"variant": 0, "threads_per_zone": 64, "zone_order": 0}),
])
def test_noalloc_matches_batch_on_two_calls(name, n1, n2, launch):
    wl = workloads.preset(name, n_zones=n1)
    say(f"case {name} launch={launch} zones={n1} then {n2}")
    net = binding.Network(wl.network)
    try:
        if launch:
            net.set_launch(**launch)
        # the second call integrates other zones (a later slice), fewer of them
        second = wl.zones.subset(np.arange(n1 - n2, n1)[::-1].copy())
        for zones in (wl.zones, second):
            want = _run(net, zones, noalloc=False)
            got = _run(net, zones, noalloc=True)
            _same(got, want)
            assert (got["zone_status"] == binding.ZONE_OK).all()
    finally:
        net.close()


def test_noalloc_single_precision_on_two_calls():
    """The single-precision kernels through the entry point that allocates nothing."""
    wl = workloads.preset("n150_r1604_arrhenius", n_zones=160)
    say("case f32 n150_r1604_arrhenius zones=160 then 48")
    net = binding.Network(wl.network)
    try:
        opts = binding.options_default(precision=binding.PREC_F32)
        second = wl.zones.subset(np.arange(100, 148))
        for zones in (wl.zones, second):
            want = _run(net, zones, noalloc=False, opts=opts)
            got = _run(net, zones, noalloc=True, opts=opts)
            _same(got, want)
            assert (got["zone_status"] == binding.ZONE_OK).all()
    finally:
        net.close()


def test_noalloc_zone_limit_and_empty_call():
    L = binding.lib()
    arr = workloads.preset("n150_r1604_arrhenius", n_zones=1)
    net = binding.Network(arr.network)
    try:
        limit = binding.NOALLOC_RATE_BYTES // (8 * arr.network.n_reactions)
        assert limit == 5066
        st = L.asy_integrate_batch_noalloc(net.handle, None, limit + 1, *([None] * 9))
        assert st == binding.ASY_EINVAL and f"at most {limit} zones" in binding.last_error()
        st = L.asy_integrate_batch_noalloc(net.handle, None, limit, *([None] * 9))
        assert st == binding.ASY_EINVAL and "non-NULL" in binding.last_error()
    finally:
        net.close()
    wl = workloads.preset("n16_r48_const", n_zones=1)
    net = binding.Network(wl.network)
    try:
        st = L.asy_integrate_batch_noalloc(net.handle, None, binding.NOALLOC_MAX_ZONES + 1,
                                           *([None] * 9))
        assert st == binding.ASY_EINVAL and "at most" in binding.last_error()
        assert L.asy_integrate_batch_noalloc(net.handle, None, 0, *([None] * 9)) == binding.ASY_OK
        o = binding.options_default(controller=binding.CTRL_LEARNED)
        st = L.asy_integrate_batch_noalloc(net.handle, C.byref(o), 1, *([None] * 9))
        assert st == binding.ASY_ESTATE   # no network weights attached
    finally:
        net.close()
