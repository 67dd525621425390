"""Pins of the MLP reference (oracle.mlp) against independent implementations."""
import numpy as np
import pytest
import torch

from oracle import mlp


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(1)
    x = np.concatenate([rng.normal(size=5000) * 10.0 ** rng.uniform(-30, 30, 5000),
                        [0.0, -0.0, 1.0, -1.0, 1.00390625, 1.005859375, 3.0e38, 1e-40]])
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16(x), want)


def _batch(seed, B=16):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-1, 1, size=(B, mlp.N_IN))
    y = rng.normal(size=B)
    return x, y


def test_backward_matches_finite_differences():
    """Central differences of the FP64 loss (rounding off) along random directions."""
    p = mlp.init_params(3)
    p[mlp.N_PARAMS - 1 - mlp.N_HID:mlp.N_PARAMS - 1] *= 50.0   # make W3 matter
    x, y = _batch(4)
    _, g = mlp.backward(p, x, y, bf16_round=False)
    rng = np.random.default_rng(5)
    for _ in range(6):
        d = rng.normal(size=mlp.N_PARAMS)
        d /= np.linalg.norm(d)
        eps = 1e-4   # truncation ~eps^2, rounding ~1e-15 * loss / eps: both far below the bound
        fd = (mlp.loss(p + eps * d, x, y, False) - mlp.loss(p - eps * d, x, y, False)) / (2 * eps)
        assert fd == pytest.approx(float(g @ d), rel=1e-6, abs=1e-9)


def test_backward_matches_torch_autograd():
    p = mlp.init_params(7)
    x, y = _batch(8, B=32)
    loss, g = mlp.backward(p, x, y, bf16_round=False)
    d = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in mlp.unpack(p).items()}
    xt = torch.zeros((32, mlp.N_IN_PAD), dtype=torch.float64)
    xt[:, :mlp.N_IN] = torch.tensor(x)
    h1 = torch.relu(xt @ d["W1"] + d["b1"])
    h2 = torch.relu(h1 @ d["W2"] + d["b2"])
    o = h2 @ d["W3"] + d["b3"][0]
    lt = torch.mean((o - torch.tensor(y)) ** 2)
    lt.backward()
    assert float(lt) == pytest.approx(loss, rel=1e-12)
    gt = np.concatenate([d[k].grad.numpy().ravel() for k in mlp.SIZES])
    np.testing.assert_allclose(g, gt, rtol=1e-10, atol=1e-14)


def test_bf16_backward_is_close_to_exact():
    p = mlp.init_params(9)
    x, y = _batch(10, B=64)
    _, g16 = mlp.backward(p, x, y, bf16_round=True)
    _, g64 = mlp.backward(p, x, y, bf16_round=False)
    assert np.linalg.norm(g16 - g64) <= 0.05 * np.linalg.norm(g64)


def test_adam_matches_torch():
    rng = np.random.default_rng(11)
    p = rng.normal(size=50)
    m = np.zeros(50)
    v = np.zeros(50)
    pt = torch.tensor(p.copy(), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([pt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 6):
        g = rng.normal(size=50)
        p, m, v = mlp.adam_step(p, g, m, v, t)
        opt.zero_grad()
        pt.grad = torch.tensor(g)
        opt.step()
    np.testing.assert_allclose(p, pt.detach().numpy(), rtol=1e-12, atol=1e-15)


def test_quantize():
    q = mlp.quantize_log2_ratio([0.0, 1.0 / 64, 3.0 / 64, -5.0, 5.0, 0.49])
    assert list(q) == [0, 0, 2, -96, 96, 16]
