"""Shared test helpers: seeded inputs, oracle states and the parity metric."""
import numpy as np
import torch

from oracle import mhd
from paper_1812_04278_amd import inputs

T64 = torch.float64


def fields(n, seed=1, v_rms=0.5, kmax=None, crop=None, B0=(1.0, 0.5, 0.0)):
    """Generator fields on an n^3 box, optionally cropped to (nx, ny, nz): the
    crop is only a way to get non-cubic, ragged-size inputs for parity tests."""
    f = inputs.random_fields(n, seed, v_rms, kmax=kmax or min(4, (n - 1) // 2), B0=B0)
    if crop is not None:
        nx, ny, nz = crop
        f.rho = np.ascontiguousarray(f.rho[:nz, :ny, :nx])
        f.v = np.ascontiguousarray(f.v[:, :nz, :ny, :nx])
        f.A = np.ascontiguousarray(f.A[:, :nz, :ny, :nx])
    return f


def oracle_state(f, h=None):
    nz, ny, nx = f.rho.shape
    cfg = mhd.Config(nx, ny, nz, h if h is not None else 1.0 / nx, gamma=f.gamma)
    return mhd.init_from_potential(f.rho, f.v, f.A, f.P0, f.B0, cfg), cfg


def rel_err(g, o):
    g = torch.as_tensor(g, dtype=T64).cpu()
    o = torch.as_tensor(o, dtype=T64).cpu()
    scale = float(o.abs().max())
    d = float((g - o).abs().max())
    return d / scale if scale > 0 else d


def state_errors(gpu, ora):
    """Normwise relative error per variable: rho, m_x, m_y, m_z, E, b_x, b_y, b_z."""
    out = {"rho": rel_err(gpu["rho"], ora["rho"]), "E": rel_err(gpu["E"], ora["E"])}
    for c, name in enumerate("xyz"):
        out["m_" + name] = rel_err(gpu["m"][c], ora["m"][c])
        out["b_" + name] = rel_err(gpu["b"][c], ora["b"][c])
    return out


def assert_state_parity(gpu, ora, tol=1e-12, label=""):
    errs = state_errors(gpu, ora)
    bad = {k: v for k, v in errs.items() if not v <= tol}
    assert not bad, f"{label} parity above {tol}: {bad}"
    return errs


def _subbox(t, centre, r):
    """Periodic sub-box of half-width r around centre (k, j, i) of [..., nz, ny, nx]."""
    k, j, i = centre
    for dim, c in ((-3, k), (-2, j), (-1, i)):
        n = t.shape[dim]
        idx = torch.tensor([(c + o) % n for o in range(-r, r)], dtype=torch.long)
        t = t.index_select(dim, idx)
    return t
