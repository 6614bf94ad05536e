"""The transpose that turns real-space gradients into gradients with respect to
the generator's Fourier amplitudes: the dot-product identity <T^T g, d> =
<g, T d> against the generator's own evaluation T (an inverse FFT written
independently), for the velocity and the three edge-staggered potential
components."""
import numpy as np
import torch

from paper_1812_04278_amd import control, inputs


def test_transpose_dot_product_identity():
    n = 12
    m = inputs.fourier_modes(seed=5, v_rms=1.0, kmax=4)
    ks = m["kset"]
    rng = np.random.default_rng(0)
    for offset in [inputs.V_OFFSET] + inputs.EDGE_OFFSETS:
        g = rng.standard_normal((n, n, n))
        da = rng.standard_normal(len(ks))
        dc = rng.standard_normal(len(ks))
        f = inputs.evaluate_modes(n, ks, da, dc, offset)            # T d
        ta, tc = control.fourier_transpose(torch.tensor(g), ks, offset)
        lhs = float((ta.numpy() * da).sum() + (tc.numpy() * dc).sum())
        rhs = float((g * f).sum())
        assert abs(lhs - rhs) <= 1e-12 * max(abs(rhs), 1.0), (offset, lhs, rhs)


def test_single_mode_by_hand():
    """g = cos(theta_k) for one mode gives dJ/da_k = n^3/2 and dJ/dc_k = 0 (and
    n^3/2 on the sine amplitude for g = sin(theta_k))."""
    n = 8
    ks = np.array([[1, 2, 0], [0, 1, 3]])
    idx = np.arange(n) + 0.5
    Z, Y, X = np.meshgrid(idx, idx, idx, indexing="ij")
    th = 2 * np.pi * (1 * X + 2 * Y) / n
    ta, tc = control.fourier_transpose(torch.tensor(np.cos(th)), ks, (0.5, 0.5, 0.5))
    np.testing.assert_allclose(ta.numpy(), [n ** 3 / 2, 0.0], atol=1e-10)
    np.testing.assert_allclose(tc.numpy(), [0.0, 0.0], atol=1e-10)
    ta, tc = control.fourier_transpose(torch.tensor(np.sin(th)), ks, (0.5, 0.5, 0.5))
    np.testing.assert_allclose(tc.numpy(), [n ** 3 / 2, 0.0], atol=1e-10)
