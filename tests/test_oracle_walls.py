"""Pins of the oracle's reflecting walls (reading R20) and floors (R21).

Walls: a closed form (a standing sound wave between two walls converges to the
exact linear solution at fifth order, which fails for a wrong mirror parity,
a missing ghost zone or a lost wall flux), conservation of mass, energy and
tangential momentum in a walled box with b_n = 0 held on the wall faces,
agreement with the periodic evolution of the mirror-doubled box, and the
cyclic relabelling of the axes.  Floors: hand-worked activations."""
import dataclasses
import math

import numpy as np
import pytest
import torch

from oracle import mhd
from paper_1812_04278_amd import inputs
from helpers import walled_state

T64 = torch.float64


def wall_faces(b, axis, n):
    return b[axis].narrow(2 - axis, n - 1, 1)


def test_walled_initial_state_is_valid():
    U, cfg = walled_state()
    assert float(wall_faces(U["b"], 0, cfg.nx).abs().max()) == 0.0
    assert float(mhd.div_faces(U["b"], cfg.h).abs().max()) < 1e-12


def test_walled_box_conserves_and_keeps_walls():
    """x walls: totals of rho, E, m_y, m_z conserved to round-off (the wall
    fluxes of these are zero by the mirror parity), b_x stays exactly zero on
    the wall faces, div_h b at round-off; m_x is not conserved (wall pressure)."""
    U0, cfg = walled_state()
    U = U0
    for _ in range(3):
        U, _ = mhd.step(U, cfg)
    for key in ("rho", "E"):
        assert abs(float(U[key].sum() - U0[key].sum())) <= 1e-13 * float(U0[key].abs().sum()), key
    for c in (1, 2):
        assert abs(float(U["m"][c].sum() - U0["m"][c].sum())) <= 1e-13 * float(U0["m"].abs().sum()), c
    assert float(wall_faces(U["b"], 0, cfg.nx).abs().max()) == 0.0
    assert float(mhd.div_faces(U["b"], cfg.h).abs().max()) < 1e-12 / cfg.h
    assert abs(float(U["m"][0].sum() - U0["m"][0].sum())) > 1e-8


def test_walled_matches_doubled_periodic_box():
    """The walled evolution equals the first half of the periodic evolution of
    the mirror-doubled box (which stays mirror symmetric), to rounding."""
    U, cfg = walled_state()
    D = mhd.mirror_double(U, 0)
    cfgD = dataclasses.replace(cfg, nx=2 * cfg.nx, walls=(False, False, False))
    dt = 0.8 * mhd.compute_dt(U, cfg)
    for _ in range(2):
        U, _ = mhd.step(U, cfg, dt)
        D, _ = mhd.step(D, cfgD, dt)
    for key in ("rho", "m", "E", "b"):
        half = D[key].narrow(D[key].dim() - 1, 0, cfg.nx)
        scale = float(U[key].abs().max())
        assert float((half - U[key]).abs().max()) <= 1e-12 * scale, key
    M = mhd.mirror_double(U, 0)
    for key in ("rho", "m", "E", "b"):
        assert float((M[key] - D[key]).abs().max()) <= 1e-12 * float(D[key].abs().max()), key


def _permute_state(U):
    """New (x, y, z) = old (z, x, y), as in the periodic permutation pin."""
    def p3(f):
        return f.permute(1, 2, 0).contiguous() if f.dim() == 3 else f.permute(0, 2, 3, 1).contiguous()
    return dict(rho=p3(U["rho"]), E=p3(U["E"]),
                m=torch.stack([p3(U["m"][2]), p3(U["m"][0]), p3(U["m"][1])]),
                b=torch.stack([p3(U["b"][2]), p3(U["b"][0]), p3(U["b"][1])]))


def test_walls_commute_with_axis_relabelling():
    """A state with x and y walls, relabelled so that the walls sit on y and z,
    steps to the relabelled result (pins the y and z walls on the x ones)."""
    U, cfg = walled_state(n=(10, 12, 8), walls=(True, True, False))
    dt = 0.01
    A, _ = mhd.step(U, cfg, dt)
    cfgP = dataclasses.replace(cfg, nx=cfg.nz, ny=cfg.nx, nz=cfg.ny, walls=(False, True, True))
    Bp, _ = mhd.step(_permute_state(U), cfgP, dt)
    PA = _permute_state(A)
    for key in U:
        assert float((PA[key] - Bp[key]).abs().max()) <= 1e-13 * float(PA[key].abs().max()), key


def standing_wave(n, t, eps=1e-6):
    """Linear standing sound wave between walls at x = 0 and 1 (B = 0, rho0 = 1,
    P0 = 0.6, gamma = 5/3, sound speed 1): rho = 1 + eps cos(pi x) cos(pi t),
    v_x = eps sin(pi x) sin(pi t), P = 0.6 + eps cos(pi x) cos(pi t); n x 1 x 1."""
    x = (torch.arange(n, dtype=T64) + 0.5) / n
    c, s = math.cos(math.pi * t), math.sin(math.pi * t)
    rho = (1.0 + eps * torch.cos(math.pi * x) * c).reshape(1, 1, n)
    vx = (eps * torch.sin(math.pi * x) * s).reshape(1, 1, n)
    P = (0.6 + eps * torch.cos(math.pi * x) * c).reshape(1, 1, n)
    m = torch.stack([rho * vx, torch.zeros_like(rho), torch.zeros_like(rho)])
    E = P / (5.0 / 3.0 - 1.0) + 0.5 * rho * vx * vx
    return dict(rho=rho, m=m, E=E, b=torch.zeros(3, 1, 1, n, dtype=T64))


def test_standing_sound_wave_fifth_order():
    """One half period (t = 1, the wave inverted) with dt ~ h^(5/3): the error of
    the fundamental -- the cos(pi x) amplitude of rho - 1 (exact: -eps) and the
    sin(pi x) amplitude of m_x (exact: 0), which nonlinearity changes only at
    O(eps^3) -- falls at fifth order (eps = 1e-5)."""
    eps = 1e-5
    errs = []
    for n in (16, 32):
        cfg = mhd.Config(n, 1, 1, 1.0 / n, walls=(True, False, False))
        U = standing_wave(n, 0.0, eps)
        nt = int(math.ceil(1.0 / (0.5 * cfg.h ** (5.0 / 3.0))))
        for _ in range(nt):
            U, _ = mhd.step(U, cfg, 1.0 / nt)
        x = (torch.arange(n, dtype=T64) + 0.5) / n
        a_rho = float(2.0 / n * ((U["rho"].flatten() - 1.0) * torch.cos(math.pi * x)).sum())
        a_m = float(2.0 / n * (U["m"][0].flatten() * torch.sin(math.pi * x)).sum())
        errs.append(abs(a_rho + eps) + abs(a_m))
    order = math.log2(errs[0] / errs[1])
    assert order > 4.5, (errs, order)


def test_floors_by_hand():
    """rho = 0.001 under rho_floor = 0.01: raised to 0.01 with m kept; a zone
    with E = 0.5, B = 0, m = 0 (P = (gamma-1) E = 1/3, below p_floor = 0.5):
    E raised by (0.5 - 1/3)/(gamma-1) so that P = 0.5; a zone with both."""
    n, g = 4, 5.0 / 3.0
    cfg = mhd.Config(n, n, n, 0.25, gamma=g, rho_floor=0.01, p_floor=0.5)
    rho = torch.ones(n, n, n, dtype=T64)
    m = torch.zeros(3, n, n, n, dtype=T64)
    E = torch.full((n, n, n), 3.0, dtype=T64)      # P = 2 elsewhere
    b = torch.zeros(3, n, n, n, dtype=T64)
    rho[1, 2, 3] = 0.001
    m[0, 1, 2, 3] = 0.0001
    E[2, 2, 2] = 0.5
    rho[3, 0, 1], E[3, 0, 1] = 0.002, 0.1
    V, nfl = mhd.apply_floors(dict(rho=rho, m=m, E=E, b=b), cfg)
    assert nfl == 4                                 # two densities, two pressures
    assert float(V["rho"][1, 2, 3]) == 0.01 and float(V["m"][0, 1, 2, 3]) == 0.0001
    _, _, _, P = mhd.primitives(V, g)
    assert abs(float(P[2, 2, 2]) - 0.5) <= 1e-15 and abs(float(P[3, 0, 1]) - 0.5) <= 1e-15
    assert float(P.min()) >= 0.5 - 1e-15
    assert abs(float(E[1, 2, 3]) - float(V["E"][1, 2, 3])) == 0.0   # P there: (3 - m^2/2rho)/.. > 0.5


def test_floors_off_is_identity_and_step_counts():
    U, cfg = walled_state(walls=(False, False, False))
    A, _ = mhd.step(U, cfg, 0.01)
    stats = {}
    B, _ = mhd.step(U, dataclasses.replace(cfg, rho_floor=1e-12, p_floor=1e-12), 0.01, stats)
    for key in U:
        assert torch.equal(A[key], B[key]), key
    assert stats.get("n_floored", 0) == 0
    # floors above the state's minima are active at every stage
    stats = {}
    hi = dataclasses.replace(cfg, rho_floor=float(U["rho"].min()) + 0.05)
    C, _ = mhd.step(U, hi, 0.01, stats)
    assert stats["n_floored"] > 0 and float(C["rho"].min()) >= hi.rho_floor
