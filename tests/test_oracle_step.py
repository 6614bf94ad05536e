"""Pins of the oracle's full step: staggered operators, CT, invariants and the
grid-aligned linear fast wave of Sect. 4.1 (closed-form solution)."""
import math

import numpy as np
import pytest
import torch

from oracle import mhd
from paper_1812_04278_amd import inputs

T64 = torch.float64
G = 5.0 / 3.0


def state(n, seed=1, v_rms=0.5, kmax=None):
    f = inputs.random_fields(n, seed, v_rms, kmax=kmax or min(4, (n - 1) // 2))
    cfg = mhd.cubic(n)
    return mhd.init_from_potential(f.rho, f.v, f.A, f.P0, f.B0, cfg), cfg


def test_interp4_exact_on_cubics():
    """B_i = (-b_{i-2} + 9 b_{i-1} + 9 b_i - b_{i+1})/16 reproduces a cubic's value
    at the zone centre from its values on faces i-3/2 .. i+3/2."""
    n = 64
    h = 1.0 / n
    xf = (torch.arange(n, dtype=T64) + 1.0) * h          # face i+1/2
    xc = (torch.arange(n, dtype=T64) + 0.5) * h          # zone i
    p = lambda x: 0.3 - 1.2 * x + 2.5 * x ** 2 - 1.7 * x ** 3
    b = p(xf).reshape(1, 1, n).expand(2, 2, n).contiguous()
    B = mhd.interp4(b, 0)[0, 0]
    # away from the periodic wrap the interpolant is exact
    np.testing.assert_allclose(B[3:-3].numpy(), p(xc)[3:-3].numpy(), rtol=0, atol=1e-14)


def test_div_curl_is_zero():
    g = torch.Generator().manual_seed(5)
    A = torch.randn(3, 6, 7, 5, generator=g, dtype=T64)
    b = mhd.curl_edges(A, 0.1)
    assert float(mhd.div_faces(b, 0.1).abs().max()) < 1e-12 * float(b.abs().max()) / 0.1


def test_ct_rhs_keeps_divergence():
    U, cfg = state(8)
    k = mhd.rhs(U, cfg)
    d = mhd.div_faces(k["b"], cfg.h)
    assert float(d.abs().max()) < 1e-12 * float(k["b"].abs().max()) / cfg.h


def test_uniform_state_preserved_bitwise():
    """A uniform state (with a Galilean boost) is an exact steady solution."""
    n = 6
    cfg = mhd.cubic(n)
    ones = torch.ones(n, n, n, dtype=T64)
    rho = 1.3 * ones
    v = torch.stack([0.7 * ones, -0.4 * ones, 0.25 * ones])
    A = torch.zeros(3, n, n, n, dtype=T64)
    U = mhd.init_from_potential(rho, v, A, 0.6, (1.0, 0.5, -0.3), cfg)
    U2, dt = mhd.step(U, cfg)
    for key in U:
        assert torch.equal(U[key], U2[key]), key


def test_conservation_and_divb():
    """Telescoping sums: totals of rho, m, E and the plane sums of each face
    component are conserved to round-off; div_h b stays at round-off."""
    U, cfg = state(12, v_rms=1.0)
    U0 = U
    for _ in range(2):
        U, _ = mhd.step(U, cfg)
    for key in ("rho", "E"):
        assert abs(float(U[key].sum() - U0[key].sum())) < 1e-12 * float(U0[key].abs().sum())
    for c in range(3):
        assert abs(float(U["m"][c].sum() - U0["m"][c].sum())) < 1e-12 * float(U0["m"].abs().sum())
    # b_x summed over each x-plane of faces (y, z), etc.
    for c, dims in ((0, (0, 1)), (1, (0, 2)), (2, (1, 2))):
        s0 = U0["b"][c].sum(dim=dims)
        s1 = U["b"][c].sum(dim=dims)
        assert float((s1 - s0).abs().max()) < 1e-12 * float(U0["b"][c].abs().sum())
    assert mhd.diagnostics(U, cfg)["max_divb"] < 1e-12 / cfg.h


def _permute_state(U):
    """Relabel axes cyclically: new (x, y, z) = old (z, x, y).  Arrays are
    [z, y, x]; the new array at [k', j', i'] is the old one at [j', i', k']."""
    def p3(f):
        return f.permute(1, 2, 0).contiguous() if f.dim() == 3 else f.permute(0, 2, 3, 1).contiguous()
    return dict(rho=p3(U["rho"]), E=p3(U["E"]),
                m=torch.stack([p3(U["m"][2]), p3(U["m"][0]), p3(U["m"][1])]),
                b=torch.stack([p3(U["b"][2]), p3(U["b"][0]), p3(U["b"][1])]))


def test_axis_permutation_symmetry():
    """Cyclically relabelling the axes of the initial state relabels the result."""
    U, cfg = state(8, v_rms=1.0)
    dt = 0.01
    A, _ = mhd.step(U, cfg, dt)
    B, _ = mhd.step(_permute_state(U), cfg, dt)
    PA = _permute_state(A)
    for key in U:
        scale = float(PA[key].abs().max())
        assert float((PA[key] - B[key]).abs().max()) < 1e-13 * scale, key


def test_ssp_rk3_amplification():
    """With a linear right-hand side k = z U / dt the step multiplies U by
    1 + z + z^2/2 + z^3/6 (increment form of the Shu-Osher scheme)."""
    U, cfg = state(4, kmax=1)
    z = -0.3
    dt = 0.1
    orig = mhd.rhs
    try:
        mhd.rhs = lambda Us, cfg: {key: (z / dt) * Us[key] for key in Us}
        U1, _ = mhd.step(U, cfg, dt)
    finally:
        mhd.rhs = orig
    amp = 1 + z + z * z / 2 + z ** 3 / 6
    for key in U:
        np.testing.assert_allclose(U1[key].numpy(), amp * U[key].numpy(), rtol=1e-14, atol=1e-15)


def _with_rhs(f, fn):
    orig = mhd.rhs
    try:
        mhd.rhs = f
        return fn()
    finally:
        mhd.rhs = orig


def test_rk4_amplification():
    """With a linear right-hand side k = z U / dt the paper's RK4 (the q_save
    accumulation of Sect. 2.1) multiplies U by the degree-4 Taylor polynomial
    of exp(z), the stability polynomial of every four-stage fourth-order RK."""
    U, cfg = state(4, kmax=1)
    z, dt = -0.7, 0.1
    U1, _ = _with_rhs(lambda Us, cfg: {key: (z / dt) * Us[key] for key in Us}, lambda: mhd.step_rk4(U, cfg, dt))
    amp = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
    for key in U:
        np.testing.assert_allclose(U1[key].numpy(), amp * U[key].numpy(), rtol=2e-15, atol=1e-15)


def _riccati(Us, cfg, c=0.8):
    return {key: c * Us[key] * Us[key] for key in Us}


def test_rk4_is_the_classical_tableau():
    """On the nonlinear autonomous ODE y' = 0.8 y^2 (zone by zone) one q_save
    step equals the textbook form of the classical RK4 -- stage slopes at
    y, y + dt/2 k1, y + dt/2 k2, y + dt k3, weights 1/6, 1/3, 1/3, 1/6 -- which
    distinguishes it from the other four-stage fourth-order methods (they share
    the linear polynomial but not this nonlinear step)."""
    U, cfg = state(4, kmax=1)
    dt = 0.05
    U1, _ = _with_rhs(_riccati, lambda: mhd.step_rk4(U, cfg, dt))
    for key in U:
        y = U[key].numpy()
        f = lambda v: 0.8 * v * v
        k1 = f(y)
        k2 = f(y + 0.5 * dt * k1)
        k3 = f(y + 0.5 * dt * k2)
        k4 = f(y + dt * k3)
        ref = y + dt / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        np.testing.assert_allclose(U1[key].numpy(), ref, rtol=1e-14, atol=1e-15)
    # a different fourth-order method (Kutta's 3/8 rule) differs at O(dt^5)
    y = U["E"].numpy()
    f = lambda v: 0.8 * v * v
    k1 = f(y)
    k2 = f(y + dt / 3 * k1)
    k3 = f(y + dt * (-k1 / 3 + k2))
    k4 = f(y + dt * (k1 - k2 + k3))
    other = y + dt / 8 * (k1 + 3 * k2 + 3 * k3 + k4)
    assert float(np.abs(other - U1["E"].numpy()).max()) > 1e3 * 1e-15 * float(np.abs(y).max())


def test_rk4_fourth_order_on_riccati():
    """y' = 0.8 y^2 has the closed form y(t) = y0 / (1 - 0.8 y0 t); the q_save
    RK4 error at t = 0.25 falls 16-fold per halving of dt."""
    U, cfg = state(4, kmax=1)
    t_end = 0.25
    errs = []
    for nt in (8, 16, 32):
        def run():
            V = U
            for _ in range(nt):
                V, _ = mhd.step_rk4(V, cfg, t_end / nt)
            return V
        V = _with_rhs(_riccati, run)
        exact = U["rho"] / (1 - 0.8 * U["rho"] * t_end)
        errs.append(float((V["rho"] - exact).abs().max()))
    orders = [math.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert all(3.8 < o < 4.2 for o in orders), (errs, orders)


# ---------------------------------------------------------------------------
# grid-aligned linear fast wave (Sect. 4.1 setup, wave vector along x)
# ---------------------------------------------------------------------------

def fast_wave_state(n, ny=1, nz=1, t=0.0, A0=1e-6):
    """Q = Qbar + A0 R_fast sin(2 pi (x - c_f t)) on an n x ny x nz box with
    h = 1/n; Qbar = (1, 0,0,0, 1, sqrt2, 1/2, E(P = 1/gamma)).  R_fast is the
    printed vector (tests/golden), c_f = 2.  Face b_y, b_z take the value at the
    x of the zone centre; b_x = 1."""
    cfg = mhd.Config(n, ny, nz, 1.0 / n)
    s5 = 1.0 / (6 * math.sqrt(5.0))
    R = [6 * s5, 12 * s5, -4 * math.sqrt(2) * s5, -2 * s5, 0.0, 8 * math.sqrt(2) * s5, 4 * s5, 27 * s5]
    x = (torch.arange(n, dtype=T64) + 0.5) / n
    s = torch.sin(2 * math.pi * (x - 2.0 * t)).reshape(1, 1, n).expand(nz, ny, n)
    Bbar = (1.0, math.sqrt(2.0), 0.5)
    Ebar = (1.0 / G) / (G - 1) + 0.5 * sum(c * c for c in Bbar)
    rho = 1.0 + A0 * R[0] * s
    m = torch.stack([A0 * R[1] * s, A0 * R[2] * s, A0 * R[3] * s])
    b = torch.stack([torch.full_like(s, 1.0), Bbar[1] + A0 * R[5] * s, Bbar[2] + A0 * R[6] * s])
    E = Ebar + A0 * R[7] * s
    return dict(rho=rho.contiguous(), m=m.contiguous(), E=E.contiguous(), b=b.contiguous()), cfg


def fast_wave_error(n, t_end, c=0.25, rk4=False):
    """L1 error of the fast wave after t_end; dt ~ h^(5/3) (SSP-RK3) or
    h^(5/4) (RK4), so that the time error falls as fast as the space error."""
    U, cfg = fast_wave_state(n)
    exact, _ = fast_wave_state(n, t=t_end)
    nt = int(math.ceil(t_end / (c * cfg.h ** (1.25 if rk4 else 5.0 / 3.0))))
    dt = t_end / nt
    for _ in range(nt):
        U, _ = (mhd.step_rk4 if rk4 else mhd.step)(U, cfg, dt)
    return mhd.l1_error(U, exact)[1]


def test_fast_wave_converges_fifth_order():
    """The scheme reduces to 1D WENO5 for a grid-aligned wave (the CT averages
    cancel), so the L1 error against the closed-form travelling wave falls as
    N^-5 with dt ~ h^(5/3) (Sect. 4.1 reports N^-5 in 1D)."""
    e = [fast_wave_error(n, 0.125) for n in (16, 32)]
    order = math.log2(e[0] / e[1])
    assert order > 4.5, (e, order)


def test_fast_wave_converges_fifth_order_rk4():
    """The same wave with the paper's RK4 and dt ~ h^(5/4), with c_f dt / h = 0.8
    at N = 32 (the paper's Courant number for RK4; 0.95 at N = 16): the error
    still falls as N^-5."""
    e = [fast_wave_error(n, 0.125, c=0.95, rk4=True) for n in (16, 32)]
    order = math.log2(e[0] / e[1])
    assert order > 4.5, (e, order)
