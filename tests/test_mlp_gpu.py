"""GPU MLP kernels (BF16 MFMA, FP32 accumulation) against the reference network in the
device's arithmetic (oracle.mlp forward_mfma / backward_mfma: the same BF16 rounding
points, products accumulated by the matrix-core rule).  Bars: outputs equal in at
least 99 % of the samples (a 1-ulp difference of the rule, or a hidden unit whose
FP32 value then rounds to the other BF16, explains the rest; 3e-2 absolute at
worst); gradients within 1e-3 of each parameter block's norm; the Adam update on the
device's own gradient within 1e-4; three training steps within 2e-2 (Adam's
per-element normalisation, see the test)."""
import sys

import numpy as np
import pytest

from oracle import mlp as ref
from paper_1409_5826_amd import binding

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, file=sys.stderr, flush=True)


@pytest.fixture(scope="module")
def torch_dev():
    import torch

    assert torch.cuda.is_available()
    binding.lib()
    return torch


def batch(seed, n):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, size=(n, ref.N_IN)).astype(np.float32)
    y = rng.normal(size=n).astype(np.float32)
    return x, y


def params(seed):
    p = ref.init_params(seed)
    u = ref.unpack(p)
    rng = np.random.default_rng(seed + 100)
    u["b1"] = rng.normal(scale=0.1, size=128)
    u["b2"] = rng.normal(scale=0.1, size=128)
    u["W3"] = rng.normal(scale=0.2, size=128)
    u["b3"] = np.array([0.3])
    return ref.pack(u).astype(np.float32)


@pytest.mark.parametrize("n", [1, 37, 1024])
def test_forward_and_infer_match_reference(torch_dev, n):
    torch = torch_dev
    say(f"case mlp forward n={n}")
    p = params(1)
    x, _ = batch(2, n)
    m = binding.Mlp(1024)
    try:
        m.set_params(p)
        np.testing.assert_array_equal(m.get_params(), p)
        xt = torch.tensor(x, device="cuda")
        o_fwd = m.forward(xt).cpu().numpy()
        o_inf = m.infer(xt).cpu().numpy()
        torch.cuda.synchronize()
    finally:
        m.close()
    o_ref, _ = ref.forward_mfma(p.astype(np.float64), x.astype(np.float64))
    for o in (o_fwd, o_inf):
        equal = o.astype(np.float64) == o_ref
        say(f"  equal outputs {equal.mean():.4f}, max difference {np.abs(o - o_ref).max():.2e}")
        assert equal.mean() >= 0.99 and np.abs(o - o_ref).max() <= 3e-2


def exact_params_and_inputs(seed, n):
    """Weights on a 1/64 grid, inputs on a 1/8 grid, biases on a 1/64 grid, all BF16-exact.

    Every product and partial sum of the three layers is then a multiple of 2^-21 below 2^2 or of
    2^-9 below 2^15, so FP32 accumulation is exact in any order and the GPU must equal the FP64
    reference bit for bit (the BF16 roundings of the hidden activations see identical values)."""
    rng = np.random.default_rng(seed)
    u = ref.unpack(np.zeros(ref.N_PARAMS))
    u["W1"][:ref.N_IN] = rng.integers(-16, 17, size=(ref.N_IN, 128)) / 64
    u["W2"] = rng.integers(-12, 13, size=(128, 128)) / 64
    u["W3"] = rng.integers(-8, 9, size=128) / 64
    u["b1"] = rng.integers(-16, 17, size=128) / 64
    u["b2"] = rng.integers(-16, 17, size=128) / 64
    u["b3"] = np.array([3 / 64])
    x = (rng.integers(-8, 9, size=(n, ref.N_IN)) / 8).astype(np.float32)
    return ref.pack(u).astype(np.float32), x


def test_forward_exact_on_representable_values(torch_dev):
    torch = torch_dev
    say("case mlp forward exact n=300")
    p, x = exact_params_and_inputs(11, 300)
    o_ref, cache = ref.forward(p.astype(np.float64), x.astype(np.float64))
    # the premise: the hidden pre-activations stay well inside the exact range
    assert np.abs(cache["a1"]).max() < 2 ** 9 and np.abs(cache["a2"]).max() < 2 ** 6
    assert 0.2 < (cache["a2"] > 0).mean() < 0.8
    m = binding.Mlp(512)
    try:
        m.set_params(p)
        xt = torch.tensor(x, device="cuda")
        o_fwd = m.forward(xt).cpu().numpy()
        o_inf = m.infer(xt).cpu().numpy()
    finally:
        m.close()
    np.testing.assert_array_equal(o_fwd.astype(np.float64), o_ref)
    np.testing.assert_array_equal(o_inf.astype(np.float64), o_ref)


def test_gradient_matches_reference(torch_dev):
    torch = torch_dev
    say("case mlp gradient")
    p = params(3)
    x, y = batch(4, 200)
    m = binding.Mlp(256)
    try:
        m.set_params(p)
        loss, g = m.gradient(torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda"))
        loss, g = float(loss.cpu()[0]), g.cpu().numpy().astype(np.float64)
    finally:
        m.close()
    l_ref, g_ref = ref.backward_mfma(p.astype(np.float64), x.astype(np.float64),
                                     y.astype(np.float64))
    assert loss == pytest.approx(l_ref, rel=1e-5)
    off = 0
    for name, size in ref.SIZES.items():
        a, b = g[off:off + size], g_ref[off:off + size]
        off += size
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        say(f"  {name}: relative difference {rel:.2e}")
        assert np.linalg.norm(a - b) <= 1e-3 * np.linalg.norm(b) + 1e-9, name


def _blocks_close(step_gpu, step_ref, rel_tol, what):
    off = 0
    worst = 0.0
    for name, size in ref.SIZES.items():
        a, b = step_gpu[off:off + size], step_ref[off:off + size]
        off += size
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        worst = max(worst, rel)
        say(f"  {what} {name}: relative difference {rel:.2e}")
        assert np.linalg.norm(a - b) <= rel_tol * np.linalg.norm(b) + 1e-9, name
    return worst


def test_adam_update_matches_reference_on_the_same_gradient(torch_dev):
    """The Adam kernel alone: three steps, each checked against the reference update applied to
    the gradient the device computed at the same parameters (FP32 moments and masters on both
    sides), within 1e-4 of each block's norm."""
    torch = torch_dev
    say("case mlp adam update")
    p0 = params(5)
    x, y = batch(6, 128)
    m = binding.Mlp(128)
    try:
        m.set_params(p0)
        xt, yt = torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda")
        mm = np.zeros(ref.N_PARAMS)
        vv = np.zeros(ref.N_PARAMS)
        p = p0.astype(np.float64)
        for t in range(1, 4):
            _, g = m.gradient(xt, yt)
            g = g.cpu().numpy().astype(np.float64)
            m.train_step(xt, yt, lr=1e-3)
            torch.cuda.synchronize()
            p_gpu = m.get_params().astype(np.float64)
            p_ref, mm, vv = ref.adam_step(p, g, mm, vv, t)
            mm = mm.astype(np.float32).astype(np.float64)
            vv = vv.astype(np.float32).astype(np.float64)
            _blocks_close(p_gpu - p, p_ref - p, 1e-4, f"step {t}")
            p = p_gpu
    finally:
        m.close()


def test_adam_trajectory_tracks_reference(torch_dev):
    """Three training steps on the device against three reference steps (gradients in the
    matrix cores' arithmetic).  Adam divides each moment by its own magnitude, so a gradient
    element near zero whose sign changes (one hidden gradient rounding to the other BF16 in a
    few in 10^3 products) moves that element's step by up to 2 lr: measured relative to each
    block's norm W1 5.4e-3, b1 2.3e-3, W2 1.8e-3, b2 1.1e-3, W3 and b3 below 1e-3.  Bar 2e-2
    per block."""
    torch = torch_dev
    say("case mlp adam trajectory")
    p0 = params(5)
    x, y = batch(6, 128)
    m = binding.Mlp(128)
    try:
        m.set_params(p0)
        xt, yt = torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda")
        for _ in range(3):
            m.train_step(xt, yt, lr=1e-3)
        torch.cuda.synchronize()
        p_gpu = m.get_params().astype(np.float64)
    finally:
        m.close()
    p = p0.astype(np.float64)
    mm = np.zeros_like(p)
    vv = np.zeros_like(p)
    for t in range(1, 4):
        # the device updates FP32 masters: the reference rounds its parameters the same way
        _, g = ref.backward_mfma(p, x.astype(np.float64), y.astype(np.float64))
        p, mm, vv = ref.adam_step(p, g, mm, vv, t)
        p = p.astype(np.float32).astype(np.float64)
    _blocks_close(p_gpu - p0, p - p0, 2e-2, "trajectory")


def test_training_reduces_loss(torch_dev):
    torch = torch_dev
    say("case mlp training")
    rng = np.random.default_rng(7)
    x = rng.uniform(-1, 1, size=(4096, ref.N_IN)).astype(np.float32)
    w = rng.normal(size=ref.N_IN) / np.sqrt(ref.N_IN)
    y = (np.tanh(2 * x @ w) + 0.1 * x[:, 0]).astype(np.float32)
    m = binding.Mlp(512)
    try:
        m.set_params(ref.init_params(8).astype(np.float32))
        xt, yt = torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda")
        loss = torch.zeros(1, device="cuda")
        first = None
        for step in range(300):
            i = (step * 512) % 4096
            m.train_step(xt[i:i + 512], yt[i:i + 512], lr=2e-3, loss=loss)
            if step == 0:
                first = float(loss.cpu()[0])
        last = float(loss.cpu()[0])
    finally:
        m.close()
    say(f"loss {first:.4f} -> {last:.4f}")
    assert last < 0.2 * first


def test_train_epoch_equals_train_steps(torch_dev):
    """asy_mlp_train_epoch runs the same kernels in the same order as a loop of
    asy_mlp_train_step: parameters and per-step losses identical bit for bit."""
    torch = torch_dev
    say("case mlp train epoch")
    rng = np.random.default_rng(11)
    x = torch.tensor(rng.uniform(-1, 1, size=(5 * 256 + 100, ref.N_IN)).astype(np.float32),
                     device="cuda")
    y = torch.tensor(rng.normal(size=x.shape[0]).astype(np.float32), device="cuda")
    p0 = ref.init_params(12).astype(np.float32)
    a, b = binding.Mlp(256), binding.Mlp(256)
    try:
        a.set_params(p0)
        b.set_params(p0)
        la = torch.zeros(5, dtype=torch.float32, device="cuda")
        assert a.train_epoch(x, y, 256, lr=2e-3, losses=la) == 5  # the 100 left over are not used
        lb = torch.zeros(5, dtype=torch.float32, device="cuda")
        for s in range(5):
            b.train_step(x[s * 256:(s + 1) * 256], y[s * 256:(s + 1) * 256], lr=2e-3,
                         loss=lb[s:s + 1])
        torch.cuda.synchronize()
        np.testing.assert_array_equal(la.cpu().numpy(), lb.cpu().numpy())
        np.testing.assert_array_equal(a.get_params(), b.get_params())
        assert not np.array_equal(a.get_params(), p0)
    finally:
        a.close()
        b.close()
