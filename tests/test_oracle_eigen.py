"""Pins of the oracle's flux, wave speeds and eigensystem (Sect. 2, Appendix A).

What fixes them, independently of the oracle's own formulas:
* the eigenvectors the paper prints for its linear-wave test (Sect. 4.1),
  stored in tests/golden/worked_example_eigenvectors.txt;
* the flux Jacobian A = dF/dq, taken by automatic differentiation of the flux:
  L A = Lambda L and A R = R Lambda;
* LAPACK eigenvalues of A against the closed-form wave speeds;
* a flux value worked out by hand from eq. (fluxes).
"""
import math
import os

import numpy as np
import pytest
import torch

from oracle import mhd

G = 5.0 / 3.0
HERE = os.path.dirname(os.path.abspath(__file__))
T64 = torch.float64


def t(x):
    return torch.as_tensor(x, dtype=T64)


def load_golden():
    out = {}
    with open(os.path.join(HERE, "golden", "worked_example_eigenvectors.txt")) as f:
        for line in f:
            line = line.split("#")[0].strip()
            if not line:
                continue
            name, scale, *ent = line.split()
            vals = []
            for e in ent:
                if e == "ig1":
                    vals.append(1.0 / (G - 1.0))
                elif e.endswith("r2"):
                    vals.append(float(e[:-2]) * math.sqrt(2.0))
                else:
                    vals.append(float(e))
            s = 1.0 / (6.0 * math.sqrt(5.0)) if scale == "s5" else float(scale)
            out[name] = np.array(vals) * s
    return out


def to8(col7):
    """7-vector (rho, m_n, m_t1, m_t2, B_t1, B_t2, E) -> 8-vector with B_x = 0 (x sweep)."""
    c = col7.tolist()
    return np.array([c[0], c[1], c[2], c[3], 0.0, c[4], c[5], c[6]])


def eig_at(rho, v, B, P):
    return mhd.eigenvectors(t(rho), t(v[0]), t(v[1]), t(v[2]), t(B[0]), t(B[1]), t(B[2]), t(P), G, 1e-30)


def test_worked_example_right_eigenvectors():
    """Sect. 4.1: R at U = (1, 0,0,0, 1, sqrt2, 1/2, 1/gamma) as printed."""
    gold = load_golden()
    B = (1.0, math.sqrt(2.0), 0.5)
    L, R = eig_at(1.0, (0, 0, 0), B, 1.0 / G)
    np.testing.assert_allclose(to8(R[:, 6]), gold["fast"], rtol=0, atol=2e-15)     # lambda = v + c_fast
    np.testing.assert_allclose(to8(R[:, 4]), gold["slow"], rtol=0, atol=2e-15)     # lambda = v + c_slow
    # the printed Alfven vector is the m = 6 column up to normalisation
    a = to8(R[:, 5])
    s = float(np.dot(a, gold["alfven"]) / np.dot(gold["alfven"], gold["alfven"]))
    np.testing.assert_allclose(a, s * gold["alfven"], rtol=0, atol=2e-15)
    # entropy mode with v_x = 1
    L, R = eig_at(1.0, (1.0, 0, 0), B, 1.0 / G)
    np.testing.assert_allclose(to8(R[:, 3]), gold["entropy"], rtol=0, atol=1e-15)
    # hydro sound wave (B = 0), right-going
    L, R = eig_at(1.0, (0, 0, 0), (0, 0, 0), 1.0 / G)
    np.testing.assert_allclose(to8(R[:, 6]), gold["sound"], rtol=0, atol=1e-15)
    L, R = eig_at(1.0, (1.0, 0, 0), (0, 0, 0), 1.0 / G)
    np.testing.assert_allclose(to8(R[:, 3]), gold["entropy"], rtol=0, atol=1e-15)


def test_worked_example_speeds():
    """The printed vectors imply c_fast = 2, c_slow = 1/2, c_A = 1 at that state."""
    cf, cA, cs = mhd.wave_speeds(t(1.0), t(1.0), t(math.sqrt(2.0)), t(0.5), t(1.0 / G), G)
    assert abs(float(cf) - 2.0) < 1e-15
    assert abs(float(cs) - 0.5) < 1e-15
    assert abs(float(cA) - 1.0) < 1e-15


def test_flux_by_hand():
    """eq. (fluxes) at rho=1, v=(1,0,0), B=(1,sqrt2,1/2), P=0.6: P* = 2.225,
    E = 3.025; F = (1, 2.225, -sqrt2, -1/2, sqrt2, 1/2, 4.25)."""
    r2 = math.sqrt(2.0)
    E = 0.6 / (G - 1) + 0.5 * (1.0 + 1.0 + 2.0 + 0.25)
    F = mhd.flux_vector(t(1.0), t(1.0), t(0.0), t(0.0), t(E), t(1.0), t(0.0), t(0.0),
                        t(1.0), t(r2), t(0.5), t(0.6))
    np.testing.assert_allclose(F.numpy(), [1.0, 2.225, -r2, -0.5, r2, 0.5, 4.25], rtol=0, atol=1e-14)


def _random_states(n, seed):
    g = torch.Generator().manual_seed(seed)
    rho = torch.rand(n, generator=g, dtype=T64) * 2 + 0.2
    v = torch.randn(3, n, generator=g, dtype=T64)
    B = torch.randn(3, n, generator=g, dtype=T64)
    P = torch.rand(n, generator=g, dtype=T64) + 0.1
    return rho, v, B, P


def _degenerate_states():
    """B_perp = 0 with c_A below and above the sound speed, B_n = 0, B = 0,
    and the triple point c_A = c_s with B_perp = 0."""
    st = []
    for Bn, Bt1, Bt2, P in [(0.5, 0.0, 0.0, 0.6), (2.0, 0.0, 0.0, 0.6), (0.0, 0.7, -0.3, 0.6),
                            (0.0, 0.0, 0.0, 0.6), (-1.0, 0.0, 0.0, 0.6), (1.0, 0.0, 0.0, 0.6)]:
        st.append((1.0, (0.3, -0.2, 0.1), (Bn, Bt1, Bt2), P))
    return st


def _flux_of_q(q, Bn):
    rho, mn, mt1, mt2, Bt1, Bt2, E = q.unbind(-1)
    vn, vt1, vt2 = mn / rho, mt1 / rho, mt2 / rho
    P = (G - 1) * (E - 0.5 * (rho * (vn ** 2 + vt1 ** 2 + vt2 ** 2) + Bn ** 2 + Bt1 ** 2 + Bt2 ** 2))
    return mhd.flux_vector(rho, mn, mt1, mt2, E, vn, vt1, vt2, Bn, Bt1, Bt2, P)


def _check_state(rho, v, B, P, tol):
    L, R = eig_at(rho, v, B, P)
    I = torch.eye(7, dtype=T64)
    E = P / (G - 1) + 0.5 * (rho * sum(x * x for x in v) + sum(x * x for x in B))
    q = t([rho, rho * v[0], rho * v[1], rho * v[2], B[1], B[2], E])
    A = torch.autograd.functional.jacobian(lambda qq: _flux_of_q(qq, t(B[0])), q)
    cf, cA, cs = mhd.wave_speeds(t(rho), t(B[0]), t(B[1]), t(B[2]), t(P), G)
    lam = mhd.eigenvalues(t(v[0]), cf, cA, cs)
    scale = 1.0 + float(A.abs().max())
    assert float((L @ R - I).abs().max()) < tol
    assert float((A @ R - R * lam).abs().max()) < tol * scale
    assert float((L @ A - lam[:, None] * L).abs().max()) < tol * scale
    # LAPACK eigenvalues of the Jacobian equal the closed-form speeds
    ev = np.sort(np.linalg.eigvals(A.numpy()).real)
    np.testing.assert_allclose(ev, np.sort(lam.numpy()), rtol=0, atol=1e-6 * scale)


def test_eigensystem_random_states():
    rho, v, B, P = _random_states(200, 1)
    for i in range(200):
        _check_state(float(rho[i]), v[:, i].tolist(), B[:, i].tolist(), float(P[i]), 1e-12)


def test_eigensystem_degenerate_states():
    for rho, v, B, P in _degenerate_states():
        _check_state(rho, v, B, P, 1e-13)


def test_eigensystem_batched_identity():
    rho, v, B, P = _random_states(20000, 2)
    L, R = mhd.eigenvectors(rho, v[0], v[1], v[2], B[0], B[1], B[2], P, G, 1e-30)
    err = (L @ R - torch.eye(7, dtype=T64)).abs().amax(dim=(-1, -2))
    cond = 1.0 + L.abs().amax(dim=(-1, -2)) * R.abs().amax(dim=(-1, -2))
    assert float((err / cond).max()) < 1e-13


def test_speed_ordering_and_textbook_form():
    """c_slow <= c_A <= c_fast, c_slow <= c_s <= c_fast, and the D form agrees with
    the textbook 1/2 (a^2 + b^2 +- sqrt((a^2 + b^2)^2 - 4 a^2 b_n^2))."""
    rho, v, B, P = _random_states(5000, 3)
    cf, cA, cs = mhd.wave_speeds(rho, B[0], B[1], B[2], P, G)
    a = torch.sqrt(G * P / rho)
    assert bool(((cs <= cA * (1 + 1e-14)) & (cA <= cf * (1 + 1e-14))).all())
    assert bool(((cs <= a * (1 + 1e-14)) & (a <= cf * (1 + 1e-14))).all())
    a2, b2, bn2 = G * P / rho, (B * B).sum(0) / rho, B[0] ** 2 / rho
    rad = torch.sqrt((a2 + b2) ** 2 - 4 * a2 * bn2)
    np.testing.assert_allclose(cf.numpy(), torch.sqrt(0.5 * (a2 + b2 + rad)).numpy(), rtol=1e-13)
    np.testing.assert_allclose((cs ** 2).numpy(), (0.5 * (a2 + b2 - rad)).numpy(),
                               rtol=0, atol=1e-12 * float((a2 + b2).max()))


def test_alpha_near_degeneracy_exact():
    """eq. (alpha) near B_perp -> 0: alpha_s^2 = (1 - (a^2 - b^2)/D)/2 is a
    difference of nearly equal terms; the eigenvectors must carry it to full
    relative precision (checked against a 50-digit evaluation of the same
    formula) and give alpha_s = 0, alpha_f = 1 exactly at B_perp = 0 with
    c_A < c_s.  R[:, 0] is the fast column (first entry alpha_f), R[:, 2] the
    slow one (first entry alpha_s)."""
    from decimal import Decimal, getcontext
    getcontext().prec = 50
    rho, P, Bn = 1.0, 0.6, 0.5
    for bp in (1e-7, 3e-5, 1e-3, 0.0):
        L, R = mhd.eigenvectors(t(rho), t(0.1), t(0.2), t(-0.3), t(Bn), t(bp), t(0.0), t(P), G, 1e-30)
        af, as_ = float(R[0, 0]), float(R[0, 2])
        a2 = Decimal(G) * Decimal(P) / Decimal(rho)
        b2 = (Decimal(Bn) ** 2 + Decimal(bp) ** 2) / Decimal(rho)
        D = ((a2 - b2) ** 2 + 4 * a2 * Decimal(bp) ** 2 / Decimal(rho)).sqrt()
        ref_s = ((1 - (a2 - b2) / D) / 2).sqrt()
        ref_f = ((1 + (a2 - b2) / D) / 2).sqrt()
        if bp == 0.0:
            assert as_ == 0.0 and af == 1.0
        else:
            assert abs(as_ / float(ref_s) - 1.0) < 1e-13, (bp, as_, float(ref_s))
            assert abs(af / float(ref_f) - 1.0) < 1e-15, (bp, af, float(ref_f))
