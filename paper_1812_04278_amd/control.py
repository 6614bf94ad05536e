"""Gradients with respect to the Fourier amplitudes of the initial fields.

The adjoint workload's control is the set of velocity and vector-potential
Fourier amplitudes that the seeded generator evaluates
(``inputs.fourier_modes``): component d of a field is
f_d(idx) = sum_k a[k, d] cos(theta_k) + c[k, d] sin(theta_k), theta_k =
2 pi k.(idx + offset)/n.  That map is linear, so the gradient of a loss J with
respect to the amplitudes is its transpose applied to dJ/df (the real-space
gradient that the rollout returns):
dJ/da[k, d] = sum_idx dJ/df_d cos(theta_k), dJ/dc[k, d] = sum_idx dJ/df_d sin(theta_k),
evaluated with one forward FFT per component.  This is control glue around
the method (no arithmetic of the scheme).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import inputs


def fourier_transpose(g: torch.Tensor, ks: np.ndarray, offset) -> tuple[torch.Tensor, torch.Tensor]:
    """(sum_idx g cos(theta_k), sum_idx g sin(theta_k)) for every mode k of ``ks``
    ([M, 3] as (kx, ky, kz)); g [nz, ny, nx] real (any device), cubic."""
    n = g.shape[-1]
    G = torch.fft.fftn(g.to(torch.float64))          # G[k] = sum_idx g exp(-2 pi i k.idx / n)
    kx = torch.as_tensor(ks[:, 0] % n, device=g.device)
    ky = torch.as_tensor(ks[:, 1] % n, device=g.device)
    kz = torch.as_tensor(ks[:, 2] % n, device=g.device)
    Gk = G[kz, ky, kx]
    ox, oy, oz = offset
    ph = torch.as_tensor(2.0 * math.pi * (ks[:, 0] * ox + ks[:, 1] * oy + ks[:, 2] * oz) / n, device=g.device)
    # sum_idx g exp(+i theta_k) = exp(i k.offset 2 pi/n) conj(G[k]) for real g
    z = torch.polar(torch.ones_like(ph), ph) * torch.conj(Gk)
    return z.real, z.imag


def amplitude_gradients(gA: torch.Tensor, gv: torch.Tensor, ks: np.ndarray) -> dict:
    """dJ/d(a_A, c_A, a_v, c_v) ([M, 3] each) from the real-space gradients
    gA = dJ/dA_edge [3, n, n, n] and gv = dJ/dv [3, n, n, n]."""
    out = {}
    for name, g, offsets in (("A", gA, inputs.EDGE_OFFSETS), ("v", gv, [inputs.V_OFFSET] * 3)):
        ca, cs = zip(*[fourier_transpose(g[d], ks, offsets[d]) for d in range(3)])
        out["a_" + name] = torch.stack(ca, dim=1)
        out["c_" + name] = torch.stack(cs, dim=1)
    return out
