"""The degenerate-face state used by the GPU parity tests: it reaches every
branch of the Appendix A renormalisation, and the oracle's eigenvectors stay a
valid basis there (L R = I at each of its face states)."""
import torch

from oracle import mhd
import pytest

from helpers import degenerate_state, face_branches, smooth_degenerate_state

STATES = [degenerate_state, smooth_degenerate_state]


@pytest.mark.parametrize("make", STATES)
def test_degenerate_state_covers_the_branches(make):
    U, cfg = make()
    c = face_branches(U, cfg)
    for k, n in c.items():
        assert n > 0, (k, c)
    assert mhd.diagnostics(U, cfg)["max_divb"] == 0.0


@pytest.mark.parametrize("make", STATES)
def test_degenerate_faces_left_right_inverse(make):
    """L R = I to 1e-13 at every face state of the three sweeps, among them the
    D = 0 triple points, B_perp = 0 with c_A on both sides of c_s, and B_n = 0."""
    U, cfg = make()
    rho, v, B, P = mhd.primitives(U, cfg.gamma)
    for axis in range(3):
        n, t1, t2 = mhd.frame(axis)
        f = lambda q: 0.5 * (q + mhd.at(q, 1, axis))
        L, R = mhd.eigenvectors(f(rho), f(v[n]), f(v[t1]), f(v[t2]), f(B[n]), f(B[t1]), f(B[t2]), f(P),
                                cfg.gamma, cfg.eps_B)
        err = (L @ R - torch.eye(7, dtype=torch.float64)).abs().max()
        assert float(err) < 1e-13, (axis, float(err))
