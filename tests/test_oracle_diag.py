"""Pins of the oracle's time step (eq. cfl), of the energy of its initial state
(eq. P) and of its diagnostics, against values worked out by hand.

Each state is built here from numbers whose consequences can be written down:
a uniform field along x gives closed-form fast speeds (c_f^2 = max(a^2, b^2)
along the field and a^2 + b^2 across it), and planted zones give known
minima, totals and divergences."""
import math

import numpy as np
import pytest
import torch

from oracle import mhd
from paper_1812_04278_amd import inputs
from helpers import diag_state

T64 = torch.float64


def conserved(rho, v, P, bface, gamma):
    """Conserved state from primitives with a face field that is uniform along
    each component's own axis (so zone B equals the face value exactly)."""
    rho = torch.as_tensor(rho, dtype=T64)
    v = torch.as_tensor(v, dtype=T64)
    b = torch.as_tensor(bface, dtype=T64)
    E = P / (gamma - 1.0) + 0.5 * rho * (v * v).sum(0) + 0.5 * (b * b).sum(0)
    return dict(rho=rho.clone(), m=(rho * v).clone(), E=E.clone(), b=b.clone())


# ---------------------------------------------------------------------------
# eq. (cfl)
# ---------------------------------------------------------------------------

def cfl_state():
    """8^3 box, gamma = 5/3, P = 0.6 (so a^2 = gamma P / rho = 1/rho), B = (2, 0, 0).

    Background rho = 1, v = 0: along x, b_n^2 = b^2 = 4 > a^2 = 1 so c_f = 2;
    across (y, z), b_n = 0 and c_f^2 = a^2 + b^2 = 5.
    Zone A (i=1, j=2, k=3): v = (0.3, 0, 0)    -> |v_x| + c_f^x = 2.3
    Zone B (i=5, j=0, k=6): v = (0, -0.7, 0)   -> |v_y| + c_f^y = 0.7 + sqrt 5
    Zone C (i=2, j=6, k=1): v = (0, 0, 0.2)    -> |v_z| + c_f^z = 0.2 + sqrt 5
    Zone D (i=7, j=7, k=7): rho = 0.64, v = 0  -> a^2 = 1.5625, b^2 = 6.25:
        c_f^x = 2.5, c_f^y = c_f^z = sqrt(7.8125)
    Maxima: x 2.5 (D), y 0.7 + sqrt 5 = 2.936 (B, beats D's 2.795), z sqrt(7.8125)
    = 2.795 (D, beats C's 2.436)."""
    n, g = 8, 5.0 / 3.0
    rho = np.ones((n, n, n))
    v = np.zeros((3, n, n, n))
    v[0, 3, 2, 1] = 0.3
    v[1, 6, 0, 5] = -0.7
    v[2, 1, 6, 2] = 0.2
    rho[7, 7, 7] = 0.64
    b = np.zeros((3, n, n, n))
    b[0] = 2.0
    cfg = mhd.Config(n, n, n, 1.0 / n, gamma=g)
    return conserved(rho, v, 0.6, b, g), cfg


def test_signal_speeds_by_hand():
    U, cfg = cfl_state()
    s = mhd.max_signal_speeds(U, cfg).numpy()
    expect = [2.5, 0.7 + math.sqrt(5.0), math.sqrt(7.8125)]
    np.testing.assert_allclose(s, expect, rtol=1e-14)


def test_dt_by_hand():
    """dt = CFL h / sum_d max(|v_d| + c_f^d): a 'max over d instead of the sum'
    gives 2.8x this, a dropped |v_d| gives sum 2.5 + 2 sqrt(5) + 2.795, a signed
    v_d (no |.|) loses zone B's 0.7 -- each differs by far more than 1e-14."""
    U, cfg = cfl_state()
    dt = mhd.compute_dt(U, cfg)
    denom = 2.5 + (0.7 + math.sqrt(5.0)) + math.sqrt(7.8125)
    assert abs(dt - 0.4 * (1.0 / 8) / denom) <= 1e-15 * dt
    wrong = {
        "max instead of sum": 0.05 / max(2.5, 0.7 + math.sqrt(5.0), math.sqrt(7.8125)),
        "dropped |v_d|": 0.05 / (2.5 + math.sqrt(5.0) + math.sqrt(7.8125)),
        "signed v_d": 0.05 / (2.5 + math.sqrt(7.8125) + math.sqrt(7.8125)),
    }
    for name, w in wrong.items():
        assert abs(w - dt) > 1e-3 * dt, name


def test_dt_isotropic_sound():
    """B = 0, rho = 1, P = 0.6, gamma = 5/3: c_f = c_s = 1 in every direction;
    with v = (0.5, -0.25, 0.125) everywhere the denominator is 1.5 + 1.25 + 1.125."""
    n, g = 5, 5.0 / 3.0
    v = np.zeros((3, n, n, n))
    v[0], v[1], v[2] = 0.5, -0.25, 0.125
    U = conserved(np.ones((n, n, n)), v, 0.6, np.zeros((3, n, n, n)), g)
    cfg = mhd.Config(n, n, n, 0.1, gamma=g, cfl=0.4)
    assert abs(mhd.compute_dt(U, cfg) - 0.04 / 3.875) <= 1e-15


# ---------------------------------------------------------------------------
# energy of the initial state (eq. P)
# ---------------------------------------------------------------------------

def test_init_energy_by_hand():
    """Uniform rho = 2, v = (0.3, -0.4, 1.2), P0 = 0.6, gamma = 5/3, A = 0,
    B0 = (1, 0.5, -0.3): E = 0.6/(2/3) + (1/2) 2 (0.09 + 0.16 + 1.44)
    + (1/2)(1 + 0.25 + 0.09) = 0.9 + 1.69 + 0.67 = 3.26; m = rho v."""
    n = 4
    cfg = mhd.cubic(n)
    ones = np.ones((n, n, n))
    v = np.stack([0.3 * ones, -0.4 * ones, 1.2 * ones])
    U = mhd.init_from_potential(2.0 * ones, v, np.zeros((3, n, n, n)), 0.6, (1.0, 0.5, -0.3), cfg)
    np.testing.assert_allclose(U["E"].numpy(), 3.26, rtol=1e-15)
    np.testing.assert_allclose(U["m"][2].numpy(), 2.4, rtol=1e-15)
    np.testing.assert_allclose(U["b"][2].numpy(), -0.3, rtol=0, atol=0)


def test_init_pressure_recovered_mach2():
    """On the random Mach-2 generator fields (v and zone B vary from zone to
    zone), the gas pressure recovered from E by eq. (P) is P0 everywhere: the
    kinetic term uses rho v^2 and the magnetic term the zone field B (the
    fourth-order interpolation of b), not the face field."""
    f = inputs.random_fields(16, seed=1, v_rms=2.0, kmax=4)
    cfg = mhd.cubic(16)
    U = mhd.init_from_potential(f.rho, f.v, f.A, f.P0, f.B0, cfg)
    _, _, _, P = mhd.primitives(U, cfg.gamma)
    assert float((P - f.P0).abs().max()) <= 1e-14 * float(U["E"].abs().max())
    # the face field differs from the zone field here: a magnetic term taken
    # from the faces would move P by far more than the bar
    b2_face = (U["b"] ** 2).sum(0)
    b2_zone = (mhd.zone_B(U["b"]) ** 2).sum(0)
    assert float((b2_face - b2_zone).abs().max()) > 1e-6


# ---------------------------------------------------------------------------
# diagnostics
# ---------------------------------------------------------------------------

def test_diagnostics_by_hand():
    U, cfg = diag_state()
    d = mhd.diagnostics(U, cfg)
    assert d["max_divb"] == 2.0 ** -7
    assert d["mass"] == 511.5
    assert d["mom"] == [0.5, 0.0, -0.25]
    assert abs(d["energy"] - (512 * 2.625 + 0.125 + 1.0 / 32 - 2.15)) <= 1e-12
    assert d["bflux"] == [512.0, 256.0 + 2.0 ** -10, 0.0]
    assert d["min_rho"] == 0.5
    assert abs(d["min_p"] - (-0.075)) <= 1e-15
    assert d["n_unphysical"] == 1


def test_diagnostics_nan_zone():
    """A NaN energy in one more zone: two unphysical zones, the minima stay those
    of the other zones (the NaN zone is reported by the count), the energy total
    is NaN and the other totals are unchanged."""
    U, cfg = diag_state()
    U["E"][1, 1, 1] = float("nan")
    d = mhd.diagnostics(U, cfg)
    assert d["n_unphysical"] == 2
    assert abs(d["min_p"] - (-0.075)) <= 1e-15
    assert d["min_rho"] == 0.5
    assert math.isnan(d["energy"])
    assert d["mass"] == 511.5
    # a NaN density: its zone's pressure is NaN too; still one zone per defect
    U["rho"][2, 3, 4] = float("nan")
    d = mhd.diagnostics(U, cfg)
    assert d["n_unphysical"] == 3 and d["min_rho"] == 0.5


def test_diagnostics_count_boundaries():
    """rho = 0 and P = 0 exactly count as unphysical (rho <= 0, P <= 0); an
    infinite energy counts too."""
    U, cfg = diag_state()
    U["E"][5, 7, 4] = 2.625                      # remove the planted negative P
    U["rho"][3, 3, 3] = 0.0
    U["E"][4, 4, 4] = 0.625                      # P = (0.625 - 0.625)/2 = 0
    U["E"][2, 2, 2] = float("inf")
    d = mhd.diagnostics(U, cfg)
    assert d["n_unphysical"] == 3, d
    assert d["min_p"] == 0.0 and d["min_rho"] == 0.0
