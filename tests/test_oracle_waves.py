"""Pins of the oblique linear-wave setup of Sect. 4.1 (3D, wave vector along
(1, 2, 2)/3 through a 2N x N x N box of size 3 x 1.5 x 1.5) and of the decay
rate of eq. (decay_rate).  The setup is checked against the closed form of a
travelling linear wave: at t = 0 the semi-discrete right-hand side must tend to
-c dQ/dx_1 = -2 pi c A0 R cos(2 pi x_1) as the grid is refined -- with the
fifth order of the WENO fluxes for the variables the mode's magnetic field does
not enter, and at least the second order of the CT field update for the rest.
A wrong rotation (a box that is not periodic along the wave) or a field
perturbation out of phase with the fluid leaves an error that does not fall."""
import math

import numpy as np
import pytest
import torch

from oracle import mhd
from paper_1812_04278_amd import inputs


def wave_state(N, mode, weights="z"):
    w = inputs.oblique_wave(N, mode)
    nz, ny, nx = w["shape"]
    cfg = mhd.Config(nx, ny, nz, w["h"], weights=weights)
    U = mhd.init_from_potential(w["rho"], np.zeros((3, nz, ny, nx)), w["A"], 0.6, w["B0"], cfg)
    U["rho"], U["m"], U["E"] = (torch.as_tensor(w[k]) for k in ("rho", "m", "E"))
    return U, cfg, w


def closed_form_rate(w, mode):
    """-c dQ/dx_1 of the travelling wave on zones (rho, m, E) and faces (b)."""
    R, c, _, _ = inputs.WAVE_MODES[mode]
    if mode == "sound":
        R = R.copy()
        R[7] = 1.0 / (w["gamma"] - 1.0)
    e1, e2, e3 = w["frame"]
    nz, ny, nx = w["shape"]
    h = w["h"]

    def x1(off):
        x = (np.arange(nx) + off[0]) * h
        y = (np.arange(ny) + off[1]) * h
        z = (np.arange(nz) + off[2]) * h
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        return e1[0] * X + e1[1] * Y + e1[2] * Z

    f = -2 * math.pi * c * 1e-6
    cz = np.cos(2 * math.pi * x1((0.5, 0.5, 0.5)))
    out = dict(rho=f * R[0] * cz, E=f * R[7] * cz,
               m=np.stack([f * (R[1] * e1[d] + R[2] * e2[d] + R[3] * e3[d]) * cz for d in range(3)]))
    face = [(1.0, 0.5, 0.5), (0.5, 1.0, 0.5), (0.5, 0.5, 1.0)]
    out["b"] = np.stack([f * (R[5] * e2[d] + R[6] * e3[d]) * np.cos(2 * math.pi * x1(face[d])) for d in range(3)])
    return out, abs(f)


def rate_errors(N, mode):
    U, cfg, w = wave_state(N, mode)
    k = mhd.rhs(U, cfg)
    ref, scale = closed_form_rate(w, mode)
    return {key: float((k[key] - torch.as_tensor(ref[key])).abs().max()) / scale for key in ref}


# mode -> (variables at fifth order, variables at >= second order)
ORDERS = {
    "fast": (("rho", "E"), ("m", "b")),
    "slow": (("rho", "E"), ("m", "b")),
    "alfven": ((), ("m", "b")),
    "entropy": (("rho", "m", "E"), ()),
    "sound": (("rho", "m", "E"), ()),
}


@pytest.mark.parametrize("mode", list(ORDERS))
def test_oblique_wave_is_the_travelling_wave(mode):
    e16, e32 = rate_errors(16, mode), rate_errors(32, mode)
    order = {k: math.log2(e16[k] / e32[k]) for k in e16 if e16[k] > 1e-7}
    hi, lo = ORDERS[mode]
    for k in hi:
        assert order[k] > 4.5, (mode, k, e16, e32, order)
    for k in lo:
        assert order[k] > 1.8, (mode, k, e16, e32, order)
    if mode in ("entropy", "sound"):    # no field perturbation: b stays put to round-off
        assert e32["b"] < 1e-7


def test_oblique_wave_setup_geometry():
    """The wave is periodic on the box, the field is divergence free and carries
    the background plus the mode's field perturbation in phase with the density."""
    e1, e2, e3 = inputs.wave_frame()
    M = np.stack([e1, e2, e3], axis=1)
    assert np.abs(M.T @ M - np.eye(3)).max() < 1e-15
    for L in ((3.0, 0, 0), (0, 1.5, 0), (0, 0, 1.5)):
        assert abs(e1 @ np.array(L) - 1.0) < 1e-15
    U, cfg, w = wave_state(16, "fast")
    assert float(mhd.div_faces(U["b"], cfg.h).abs().max()) < 1e-12
    B = mhd.zone_B(U["b"])
    Bw2 = sum(B[d] * e2[d] for d in range(3)) - math.sqrt(2.0)
    drho = U["rho"] - 1.0
    R = inputs.WAVE_MODES["fast"][0]
    # zone field perturbation = (R_B2 / R_rho) x density perturbation (fourth-order
    # interpolation from the faces: exact to O(h^4) relative)
    assert float((Bw2 - R[5] / R[0] * drho).abs().max()) < 1e-2 * 1e-6 * abs(R[5])


def test_decay_rate_closed_form():
    """A field fluctuation that decays as exp(-0.3 t) has tau_D = 0.3; the rms of
    the wave's transverse field at t = 0 is A0 |R_B2| / sqrt(2) up to O(h^2):
    the faces hold face averages of B (the curl of A through each face)."""
    U, cfg, w = wave_state(16, "fast")
    e2 = w["frame"][1]
    r0 = mhd.wave_rms(U, e2, math.sqrt(2.0))
    R = inputs.WAVE_MODES["fast"][0]
    assert abs(r0 / (1e-6 * abs(R[5]) / math.sqrt(2.0)) - 1.0) < 2e-2
    B0 = torch.tensor(w["B0"], dtype=torch.float64).reshape(3, 1, 1, 1)
    Ut = dict(U)
    Ut["b"] = B0 + (U["b"] - B0) * math.exp(-0.3 * 2.0)
    # the fluctuation is 4e-7 of the field: field rounding enters its rms at ~1e-10
    assert abs(mhd.decay_rate(r0, mhd.wave_rms(Ut, e2, math.sqrt(2.0)), 2.0) - 0.3) < 1e-8
