"""Host-side checks of the C-ABI library: it loads, exports every declared
symbol, and rejects invalid descriptors and options before any device call.
No GPU is needed (and none is used for compute)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_1409_5826_amd import binding, workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "asynet.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(asy_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    L = binding.lib()
    syms = declared_symbols()
    assert len(syms) >= 9
    for s in syms:
        assert hasattr(L, s), s
    assert set(syms) == set(binding.EXPORTS)


def test_options_default():
    o = binding.options_default()
    assert (o.kappa, o.tol, o.y_floor, o.grow_max, o.safety, o.shrink_min, o.dt_min) == \
        (1.0, 0.01, 1e-10, 2.0, 0.9, 0.1, 1e-20)
    assert o.max_steps == 10_000_000 and o.controller == binding.CTRL_PLAIN
    assert o.precision == binding.PREC_F64


def _create(**kw):
    net = workloads.preset("n16_r48_const", n_zones=1).network
    args = dict(n_species=net.n_species, reactant0=net.reactant0.copy(),
                reactant1=net.reactant1.copy(), product=net.product.copy(), weight=net.weight.copy())
    args.update(kw)
    return binding.asy_network_create(**args)


def _expect_einval(**kw):
    with pytest.raises(binding.AsyError) as ei:
        _create(**kw)
    assert ei.value.status == binding.ASY_EINVAL, str(ei.value)
    return str(ei.value)


def test_descriptor_validation():
    net = workloads.preset("n16_r48_const", n_zones=1).network
    r0, r1, pr, w = net.reactant0, net.reactant1, net.product, net.weight
    two = int(np.flatnonzero(r1 >= 0)[0])
    one = int(np.flatnonzero(r1 < 0)[0])
    bad = r0.copy(); bad[3] = 16
    assert "out of range" in _expect_einval(reactant0=bad)
    bad = r1.copy(); bad[two] = r0[two]
    assert "identical reactants" in _expect_einval(reactant1=bad)
    bad = pr.copy(); bad[one] = r0[one]
    assert "product equals a reactant" in _expect_einval(product=bad)
    bad = w.copy(); bad[pr[two]] += 1
    assert "conserve weight" in _expect_einval(weight=bad)
    bad = r1.copy(); bad[one] = -2
    assert "out of range" in _expect_einval(reactant1=bad)
    _expect_einval(n_species=0)
    R = len(r0)
    assert "Arrhenius" in _expect_einval(A=np.full(R, -1.0), E=np.zeros(R))
    _expect_einval(A=np.full(R, np.nan), E=np.zeros(R))
    _expect_einval(A=np.ones(R), E=np.full(R, np.inf))
    assert "split_above" in _expect_einval(split_above=5)
    assert "split_above" in _expect_einval(split_above=-1)


def test_valid_descriptor_needs_a_device():
    """A valid descriptor passes validation and stops at the device check here."""
    import torch

    if torch.cuda.is_available():
        pytest.skip("a device is present")
    with pytest.raises(binding.AsyError) as ei:
        _create()
    assert ei.value.status == binding.ASY_EDEVICE


def test_null_arguments():
    L = binding.lib()
    assert L.asy_network_create(None, None) == binding.ASY_EINVAL
    assert L.asy_integrate_batch(None, None, 0, *([None] * 9)) == binding.ASY_EINVAL
    assert L.asy_get_launch(None, None) == binding.ASY_EINVAL
    L.asy_network_destroy(None)   # no-op
    assert binding.asy_version().startswith("asynet")


def test_layout_info_argument_errors():
    L = binding.lib()
    info = binding.asy_layout_info()
    assert L.asy_network_layout_info(None, 128, C.byref(info)) == binding.ASY_EINVAL


def test_single_precision_rejects_a_subnormal_y_floor():
    """Options are validated before anything else: in single precision y_floor is rounded
    to float, so a value below the smallest normal float is refused."""
    L = binding.lib()
    for floor, ok in ((1e-39, False), (0.0, False), (1.1754943508222875e-38, True), (1e-30, True)):
        o = binding.options_default(precision=binding.PREC_F32, y_floor=floor)
        st = L.asy_integrate_batch(None, C.byref(o), 0, *([None] * 9))
        assert st == binding.ASY_EINVAL
        msg = binding.last_error()
        assert ("y_floor" in msg) != ok, (floor, msg)
    o = binding.options_default(y_floor=1e-300)  # double precision keeps any positive floor
    assert L.asy_integrate_batch(None, C.byref(o), 0, *([None] * 9)) == binding.ASY_EINVAL
    assert "net" in binding.last_error()
