"""Host-side parts of the learned-controller pipeline (no GPU)."""
import numpy as np

from paper_1409_5826_amd import binding, learned


def test_initial_params_layout():
    p = learned.initial_params(3)
    assert p.dtype == np.float32 and p.shape == (binding.MLP_N_PARAMS,)
    w1 = p[:192 * 128].reshape(192, 128)
    assert (w1[166:] == 0).all() and np.abs(w1[:166]).max() <= np.sqrt(6 / 166)
    b1 = p[192 * 128:192 * 128 + 128]
    assert (b1 == 0).all() and p[-1] == 0
    np.testing.assert_array_equal(p, learned.initial_params(3))
    assert not np.array_equal(p, learned.initial_params(4))


def test_mass_error():
    Y = np.array([[1.0, 2.0], [0.5, 0.5]])
    R = np.array([[1.0, 1.0], [1.0, 0.5]])
    np.testing.assert_allclose(learned.mass_error(Y, R, np.array([1, 3])), [3.0, 0.5])


def test_step_scale_augmentation_shifts_step_features_and_labels():
    """A record for a last step h 2^d: the step features move by d log10(2)/10, the label by -d
    (clipped to +-3); abundances and the tolerance feature do not move."""
    import torch

    n = 5
    x = torch.zeros((2, binding.MLP_N_IN), dtype=torch.float32)
    x[:, :n] = -0.5
    x[:, n:n + 3] = torch.tensor([-0.2, -0.4, -0.6])
    x[:, n + 3] = -0.2
    tr = learned.Traces(x=x, y=torch.tensor([0.1, -2.5]), zone=np.array([3, 4]),
                        n_acc=np.array([10, 20]), taken=2)
    out = learned.augment_step_scale(tr, n, shifts=(-4, 1))
    assert out.x.shape == (6, binding.MLP_N_IN) and len(out.zone) == 6
    np.testing.assert_array_equal(out.zone, [3, 4, 3, 4, 3, 4])
    s = np.log10(2.0) / 10
    np.testing.assert_allclose(out.x[2:4, n:n + 3].numpy(), x[:, n:n + 3].numpy() - 4 * s, atol=1e-6)
    np.testing.assert_allclose(out.x[4:6, n:n + 3].numpy(), x[:, n:n + 3].numpy() + s, atol=1e-6)
    np.testing.assert_array_equal(out.x[2:, :n].numpy(), -0.5)
    np.testing.assert_array_equal(out.x[2:, n + 3].numpy(), np.float32(-0.2))
    np.testing.assert_allclose(out.y.numpy(), [0.1, -2.5, 3.0, 1.5, -0.9, -3.0], atol=1e-6)
