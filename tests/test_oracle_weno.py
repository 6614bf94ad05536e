"""Pins of the oracle's WENO5 flux (Sect. 2.2, eq. FWENO).

* The difference form of eq. (FWENO) with phi_N equals the textbook three-stencil
  Jiang-Shu reconstruction (candidate parabolas + smoothness indicators beta_k)
  with epsilon/12, since IS_k = 12 beta_k.  The textbook form is written here
  from its own definition, not from the oracle's code.
* With epsilon -> infinity the weights become the linear ones and the flux is the
  linear fifth-order upwind flux (2, -13, 47, 27, -3)/60.
* A 1D scalar advection run with the oracle's split flux converges at 5th order.
* WENO-Z (reading R13: alpha_k = d_k (1 + (tau_5 / (eps_Z + IS_k))^2)) equals the
  textbook WENO-Z reconstruction of Borges, Carmona, Costa & Don (2008) with the
  exponent 2 and eps_Z/12 (the ratio tau_5/IS_k is unchanged by the factor 12),
  written here from its own definition; with eps_Z -> infinity it is the linear
  upwind flux; and it advects at 5th order.
* WENO-Z as Sect. 2.2 prints it, alpha_k = d_k (1 + tau_5 / (eps_Z + IS_k)^2): on
  data scaled to tau_5 = 1 it equals the reading R13 pinned above; its excess
  tau_5 / IS_k^2 has the dimension 1/IS, so scaling the data by s moves phi_N(s v)/s
  towards the linear-weight value as s^-2 (R13: not at all); and as s -> 0 the
  weights tend to d_k / IS_k^2, the Jiang-Shu weights with eps -> 0.
"""
import math

import numpy as np
import torch

from oracle import mhd

T64 = torch.float64


def textbook_js_plus(f, eps):
    """Left-biased WENO5-JS value at i+1/2 from f_{i-2..i+2} (Jiang & Shu 1996)."""
    fm2, fm1, f0, fp1, fp2 = f
    q0 = (2 * fm2 - 7 * fm1 + 11 * f0) / 6
    q1 = (-fm1 + 5 * f0 + 2 * fp1) / 6
    q2 = (2 * f0 + 5 * fp1 - fp2) / 6
    b0 = 13 / 12 * (fm2 - 2 * fm1 + f0) ** 2 + 0.25 * (fm2 - 4 * fm1 + 3 * f0) ** 2
    b1 = 13 / 12 * (fm1 - 2 * f0 + fp1) ** 2 + 0.25 * (fm1 - fp1) ** 2
    b2 = 13 / 12 * (f0 - 2 * fp1 + fp2) ** 2 + 0.25 * (3 * f0 - 4 * fp1 + fp2) ** 2
    a0, a1, a2 = 0.1 / (eps + b0) ** 2, 0.6 / (eps + b1) ** 2, 0.3 / (eps + b2) ** 2
    s = a0 + a1 + a2
    return (a0 * q0 + a1 * q1 + a2 * q2) / s


def textbook_z_plus(f, eps):
    """Left-biased WENO5-Z value at i+1/2 from f_{i-2..i+2} (Borges et al. 2008, exponent 2)."""
    fm2, fm1, f0, fp1, fp2 = f
    q0 = (2 * fm2 - 7 * fm1 + 11 * f0) / 6
    q1 = (-fm1 + 5 * f0 + 2 * fp1) / 6
    q2 = (2 * f0 + 5 * fp1 - fp2) / 6
    b0 = 13 / 12 * (fm2 - 2 * fm1 + f0) ** 2 + 0.25 * (fm2 - 4 * fm1 + 3 * f0) ** 2
    b1 = 13 / 12 * (fm1 - 2 * f0 + fp1) ** 2 + 0.25 * (fm1 - fp1) ** 2
    b2 = 13 / 12 * (f0 - 2 * fp1 + fp2) ** 2 + 0.25 * (3 * f0 - 4 * fp1 + fp2) ** 2
    tau = (b0 - b2).abs()
    a0 = 0.1 * (1 + (tau / (b0 + eps)) ** 2)
    a1 = 0.6 * (1 + (tau / (b1 + eps)) ** 2)
    a2 = 0.3 * (1 + (tau / (b2 + eps)) ** 2)
    s = a0 + a1 + a2
    return (a0 * q0 + a1 * q1 + a2 * q2) / s


def split_values(seed, n, smooth):
    g = torch.Generator().manual_seed(seed)
    if smooth:
        x = torch.linspace(0, 1, 6, dtype=T64)[:, None]
        ph = torch.rand(1, n, generator=g, dtype=T64) * 6.28
        amp = torch.rand(1, n, generator=g, dtype=T64)
        return amp * torch.sin(2 * math.pi * 0.3 * x + ph)
    return torch.randn(6, n, generator=g, dtype=T64) * torch.rand(1, n, generator=g, dtype=T64) * 3


def test_phiN_equals_textbook_js():
    cfg = mhd.Config(4, 4, 4, 0.25)
    for smooth in (False, True):
        fp = split_values(1, 5000, smooth)            # f^+ on zones i-2..i+3
        fmv = split_values(2, 5000, smooth)           # f^- on zones i-2..i+3
        # the oracle's characteristic flux is built from F^s and q^s with F^+- = (F +- alpha q)/2;
        # choose F = f^+ + f^-, q = f^+ - f^- and alpha = 1
        Fs = [fp[k] + fmv[k] for k in range(6)]
        qs = [fp[k] - fmv[k] for k in range(6)]
        got = mhd.weno_split_flux(Fs, qs, torch.ones(()), cfg)
        plus = textbook_js_plus([fp[k] for k in range(0, 5)], cfg.eps / 12)
        minus = textbook_js_plus([fmv[k] for k in range(5, 0, -1)], cfg.eps / 12)   # mirrored stencil
        ref = plus + minus
        np.testing.assert_allclose(got.numpy(), ref.numpy(), rtol=0, atol=2e-14 * (1 + float(ref.abs().max())))


def test_linear_limit_is_upwind5():
    cfg = mhd.Config(4, 4, 4, 0.25, eps=1e30)
    g = torch.Generator().manual_seed(3)
    f = torch.randn(6, 1000, generator=g, dtype=T64)
    Fs = [f[k] for k in range(6)]
    qs = [f[k] for k in range(6)]           # alpha = 1: F^+ = F, F^- = 0
    got = mhd.weno_split_flux(Fs, qs, torch.ones(()), cfg)
    ref = (2 * f[0] - 13 * f[1] + 47 * f[2] + 27 * f[3] - 3 * f[4]) / 60
    np.testing.assert_allclose(got.numpy(), ref.numpy(), rtol=0, atol=1e-14)


def _advect(n, t_end, cfl=0.4, weights="js"):
    """u_t + u_x = 0 on [0,1), f(u) = u, alpha = 1, SSP-RK3, dt ~ h^(5/3)."""
    cfg = mhd.Config(n, 1, 1, 1.0 / n, weights=weights)
    h = 1.0 / n
    x = (torch.arange(n, dtype=T64) + 0.5) * h
    u0 = torch.sin(2 * math.pi * x)
    dt_target = cfl * h ** (5.0 / 3.0)
    nt = int(math.ceil(t_end / dt_target))
    dt = t_end / nt

    def L(u):
        st = [torch.roll(u, -o) for o in range(-2, 4)]
        F = mhd.weno_split_flux(st, st, torch.ones(()), cfg)
        return -(F - torch.roll(F, 1)) / h
    u = u0.clone()
    for _ in range(nt):
        u1 = u + dt * L(u)
        u2 = 0.75 * u + 0.25 * (u1 + dt * L(u1))
        u = u / 3 + 2.0 / 3.0 * (u2 + dt * L(u2))
    exact = torch.sin(2 * math.pi * (x - t_end))
    return float((u - exact).abs().mean())


def test_scalar_advection_fifth_order():
    e = [_advect(n, 0.5) for n in (20, 40, 80)]
    orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert orders[-1] > 4.6, (e, orders)


def test_lax_friedrichs_speed_bounds_both_zones():
    """alpha(m) on face i+1/2 is the larger |lambda(m)| of zones i and i+1, so
    both split fluxes are monotone across the face (Sect. 2.2)."""
    g = torch.Generator().manual_seed(7)
    for axis in range(3):
        lam = torch.randn(5, 6, 7, 7, generator=g, dtype=T64)
        a = mhd.lf_speed(lam, axis)
        nxt = mhd.at(lam.movedim(-1, 0), 1, axis).movedim(0, -1)
        assert bool((a >= lam.abs()).all()) and bool((a >= nxt.abs()).all())
        assert bool(((a == lam.abs()) | (a == nxt.abs())).all())


def test_phiN_wenoz_equals_textbook_z():
    cfg = mhd.Config(4, 4, 4, 0.25, weights="z", eps_Z=1e-12)
    for smooth in (False, True):
        fp = split_values(11, 5000, smooth)
        fmv = split_values(12, 5000, smooth)
        Fs = [fp[k] + fmv[k] for k in range(6)]
        qs = [fp[k] - fmv[k] for k in range(6)]
        got = mhd.weno_split_flux(Fs, qs, torch.ones(()), cfg)
        ref = textbook_z_plus([fp[k] for k in range(0, 5)], cfg.eps_Z / 12) + \
            textbook_z_plus([fmv[k] for k in range(5, 0, -1)], cfg.eps_Z / 12)
        np.testing.assert_allclose(got.numpy(), ref.numpy(), rtol=0, atol=2e-14 * (1 + float(ref.abs().max())))
    # and with the paper's eps_Z = 1e-40, including constant stencils (tau_5 = IS_k = 0)
    cfg = mhd.Config(4, 4, 4, 0.25, weights="z")
    f = split_values(13, 2000, True)
    f[:, :100] = 0.7
    Fs = [f[k] for k in range(6)]
    got = mhd.weno_split_flux(Fs, Fs, torch.ones(()), cfg)
    ref = textbook_z_plus([f[k] for k in range(0, 5)], cfg.eps_Z / 12)
    assert bool(torch.isfinite(got).all())
    np.testing.assert_allclose(got.numpy(), ref.numpy(), rtol=0, atol=2e-14 * (1 + float(ref.abs().max())))


def test_wenoz_linear_limit_is_upwind5():
    cfg = mhd.Config(4, 4, 4, 0.25, weights="z", eps_Z=1e30)
    g = torch.Generator().manual_seed(14)
    f = torch.randn(6, 1000, generator=g, dtype=T64)
    Fs = [f[k] for k in range(6)]
    got = mhd.weno_split_flux(Fs, Fs, torch.ones(()), cfg)
    ref = (2 * f[0] - 13 * f[1] + 47 * f[2] + 27 * f[3] - 3 * f[4]) / 60
    np.testing.assert_allclose(got.numpy(), ref.numpy(), rtol=0, atol=1e-14)


def test_wenoz_scalar_advection_fifth_order():
    e = [_advect(n, 0.5, weights="z") for n in (20, 40, 80)]
    orders = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert orders[-1] > 4.6, (e, orders)


def _phi_cfgs():
    z = mhd.Config(4, 4, 4, 0.25, weights="z")
    return z, mhd.Config(4, 4, 4, 0.25, weights="z_printed")


def _stencils(seed, n=4000):
    g = torch.Generator().manual_seed(seed)
    return torch.randn(4, n, generator=g, dtype=T64)


def test_wenoz_printed_equals_reading_at_unit_tau():
    z, zp = _phi_cfgs()
    a, b, c, d = _stencils(21)
    IS0 = 13 * (a - b) ** 2 + 3 * (a - 3 * b) ** 2
    IS2 = 13 * (c - d) ** 2 + 3 * (3 * c - d) ** 2
    s = 1.0 / torch.sqrt((IS0 - IS2).abs())   # IS is quadratic in the data: tau_5(s v) = 1
    v = [x * s for x in (a, b, c, d)]
    ref = mhd.phi_N(*v, z)
    got = mhd.phi_N(*v, zp)
    np.testing.assert_allclose(got.numpy(), ref.numpy(), rtol=0, atol=1e-13 * (1 + float(ref.abs().max())))
    # away from unit tau_5 the two forms differ
    assert float((mhd.phi_N(*(4 * x for x in v), zp) / 4 - ref).abs().max()) > 1e-3


def test_wenoz_printed_scale_rate():
    z, zp = _phi_cfgs()
    lin = mhd.Config(4, 4, 4, 0.25, weights="js", eps=1e30)   # linear weights (pinned above)
    a, b, c, d = _stencils(22)
    ref = mhd.phi_N(a, b, c, d, lin)

    def dev(cfg, s):
        return (mhd.phi_N(s * a, s * b, s * c, s * d, cfg) / s - ref).abs()

    rate = torch.log10(dev(zp, 1e3) / dev(zp, 1e4))
    assert abs(float(rate.median()) - 2.0) < 0.01, float(rate.median())
    rate_z = torch.log10(dev(z, 1e3) / dev(z, 1e4))
    assert abs(float(rate_z.median())) < 0.01   # the reading R13 is scale-invariant


def test_wenoz_printed_small_scale_is_js_without_eps():
    _, zp = _phi_cfgs()
    js0 = mhd.Config(4, 4, 4, 0.25, weights="js", eps=1e-35)
    a, b, c, d = _stencils(23)
    s = 1e-8
    got = mhd.phi_N(s * a, s * b, s * c, s * d, zp) / s
    ref = mhd.phi_N(s * a, s * b, s * c, s * d, js0) / s
    np.testing.assert_allclose(got.numpy(), ref.numpy(), rtol=0, atol=1e-9 * (1 + float(ref.abs().max())))


def test_wenoz_printed_constant_stencils_are_linear():
    _, zp = _phi_cfgs()
    f = split_values(13, 2000, True)
    f[:, :100] = 0.7
    Fs = [f[k] for k in range(6)]
    got = mhd.weno_split_flux(Fs, Fs, torch.ones(()), zp)
    ref = (2 * f[0] - 13 * f[1] + 47 * f[2] + 27 * f[3] - 3 * f[4]) / 60
    assert bool(torch.isfinite(got).all())
    np.testing.assert_allclose(got[:100].numpy(), ref[:100].numpy(), rtol=0, atol=1e-14)
