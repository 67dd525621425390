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
