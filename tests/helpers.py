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


# ---------------------------------------------------------------------------
# a state on the degeneracies of the Appendix A eigensystem (slab layout in
# tests/test_gpu_degenerate.py)
# ---------------------------------------------------------------------------

GAMMA = 2.0
SHAPE = (18, 20, 72)          # nz, ny, nx
AMP = [0.0, 0.0, 0.0, 1e-16, 1e-7, 1e-5, 1e-3, 0.3]
PRES = [0.5, 0.3, 0.8, 0.6, 0.6, 0.6, 0.6, 0.6]


def degenerate_state():
    """The slab state described in tests/test_gpu_degenerate.py, as the oracle's
    conserved dict, and its configuration (gamma = 2)."""
    nz, ny, nx = SHAPE
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    z = (np.arange(nz) + 0.5) / nz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    slab = np.minimum(np.arange(nx) // 9, 7)
    amp = np.array(AMP)[slab][None, None, :]
    pres = np.array(PRES)[slab][None, None, :] * np.ones(SHAPE)
    rho = 1.0 + 0.15 * np.sin(2 * np.pi * (2 * X + Y) + 0.3) + 0.1 * np.cos(2 * np.pi * (Z - X) + 1.1)
    vx = 0.3 * np.sin(2 * np.pi * (X + 2 * Y + Z) + 0.7)
    vy = 0.2 * np.cos(2 * np.pi * (3 * X - Z) + 0.2)
    vz = 0.25 * np.sin(2 * np.pi * (Y + X) + 1.9)
    v = np.stack([vx, vy, vz])
    v[:, :, :, slab == 0] = 0.0                  # static D = 0 slab
    v[1:, :, :, (slab == 1) | (slab == 2)] = 0.0  # longitudinal flow keeps B_perp = 0
    b = np.zeros((3,) + SHAPE)
    b[0] = 1.0
    b[1] = amp * np.cos(2 * np.pi * Z + 0.4) * np.ones(SHAPE)      # b_y(x, z)
    b[2] = amp * np.sin(2 * np.pi * Y + 1.1) * np.ones(SHAPE)      # b_z(x, y)
    # zone B equals the face values here (b_t is uniform along its own axis)
    E = pres / (GAMMA - 1.0) + 0.5 * rho * (v * v).sum(0) + 0.5 * (b * b).sum(0)
    U = dict(rho=torch.tensor(rho), m=torch.tensor(rho * v), E=torch.tensor(E), b=torch.tensor(b))
    cfg = mhd.Config(nx, ny, nz, 1.0 / nx, gamma=GAMMA)
    return U, cfg


def smooth_degenerate_state():
    """The slab state with cosine ramps over the four zones around each slab edge
    (the slab interiors, zones 2..6 of each, keep the exact values: D = 0, B_perp
    = 0, B_perp^2 below eps_B, ...), so the data are smooth at the slab edges."""
    nz, ny, nx = SHAPE
    x = (np.arange(nx) + 0.5) / nx; y = (np.arange(ny) + 0.5) / ny; z = (np.arange(nz) + 0.5) / nz
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    i = np.arange(nx); s = np.minimum(i // 9, 7); r = i % 9
    w_prev = np.where(r < 2, 0.5 * (1 - np.sin(np.pi * (r + 0.5) / 4)), 0.0)     # weight of previous slab
    w_next = np.where(r > 6, 0.5 * (1 - np.sin(np.pi * (8.5 - r) / 4)), 0.0)
    sp = (s - 1) % 8; sn = (s + 1) % 8
    def blend(vals):
        vals = np.asarray(vals)
        return (1 - w_prev - w_next) * vals[s] + w_prev * vals[sp] + w_next * vals[sn]
    amp = blend(AMP)[None, None, :]; pres = blend(PRES)[None, None, :] * np.ones(SHAPE)
    mv0 = blend([0, 1, 1, 1, 1, 1, 1, 1]); mvt = blend([0, 0, 0, 1, 1, 1, 1, 1])
    rho = 1.0 + 0.15 * np.sin(2 * np.pi * (2 * X + Y) + 0.3) + 0.1 * np.cos(2 * np.pi * (Z - X) + 1.1)
    vx = 0.3 * np.sin(2 * np.pi * (X + 2 * Y + Z) + 0.7) * mv0
    vy = 0.2 * np.cos(2 * np.pi * (3 * X - Z) + 0.2) * mvt
    vz = 0.25 * np.sin(2 * np.pi * (Y + X) + 1.9) * mvt
    v = np.stack([vx, vy, vz])
    b = np.zeros((3,) + SHAPE); b[0] = 1.0
    b[1] = amp * np.cos(2 * np.pi * Z + 0.4) * np.ones(SHAPE)
    b[2] = amp * np.sin(2 * np.pi * Y + 1.1) * np.ones(SHAPE)
    E = pres / (GAMMA - 1.0) + 0.5 * rho * (v * v).sum(0) + 0.5 * (b * b).sum(0)
    U = dict(rho=torch.tensor(rho), m=torch.tensor(rho * v), E=torch.tensor(E), b=torch.tensor(b))
    return U, mhd.Config(nx, ny, nz, 1.0 / nx, gamma=GAMMA)


def face_branches(U, cfg):
    """Counts of x faces on each branch and of y faces with B_n = 0 or tiny, from
    the oracle's primitives (to show that the state exercises every branch)."""
    rho, v, Bz, P = mhd.primitives(U, cfg.gamma)
    f = lambda q, ax: 0.5 * (q + mhd.at(q, 1, ax))
    r, p = f(rho, 0), f(P, 0)
    Bn, Bt1, Bt2 = f(Bz[0], 0), f(Bz[1], 0), f(Bz[2], 0)
    a2 = cfg.gamma * p / r
    b2 = (Bn * Bn + Bt1 * Bt1 + Bt2 * Bt2) / r
    bp2 = Bt1 * Bt1 + Bt2 * Bt2
    D = torch.sqrt((a2 - b2) ** 2 + 4.0 * a2 * bp2 / r)
    By_face = f(Bz[1], 1)
    return dict(
        D_zero=int((D == 0).sum()),
        Bperp_zero=int((bp2 == 0).sum()),
        Bperp_below_epsB=int(((bp2 > 0) & (bp2 <= cfg.eps_B)).sum()),
        Bperp_small=int(((bp2 >= 1e-15) & (bp2 <= 1e-5)).sum()),
        y_Bn_zero=int((By_face == 0).sum()),
        y_Bn_tiny_pos=int(((By_face > 0) & (By_face < 1e-6)).sum()),
        y_Bn_tiny_neg=int(((By_face < 0) & (By_face > -1e-6)).sum()),
    )


def diag_state():
    """8^3 box, gamma = 1.5 (gamma - 1 = 1/2 exactly), h = 1/8.

    Background: rho = 1, v = 0, P = 1, face b = (1, 1/2, 0), so zone B = (1, 1/2, 0)
    and E = 2 + 0.625 = 2.625.  Planted:
      zone (i=3, j=5, k=6): rho = 1/2                     (min rho = 0.5)
      zone (i=0, j=0, k=0): m_x = 1/2 with E = 2.75       (P = 1 still)
      zone (i=6, j=6, k=2): m_z = -1/4, E = 2.625 + 1/32  (P = 1 still)
      zone (i=4, j=7, k=5): E = 0.475                     (P = (0.475 - 0.625)/2 = -0.075)
      face b_y at (i=1, j=2, k=1) += 2^-10                (div = +-2^-10 / h = +-2^-7)
    Totals: mass 511.5, m = (1/2, 0, -1/4), E = 512 * 2.625 + 0.125 + 1/32 - 2.15,
    b = (512, 256 + 2^-10, 0)."""
    n, g = 8, 1.5
    rho = torch.ones(n, n, n, dtype=T64)
    m = torch.zeros(3, n, n, n, dtype=T64)
    E = torch.full((n, n, n), 2.625, dtype=T64)
    b = torch.zeros(3, n, n, n, dtype=T64)
    b[0], b[1] = 1.0, 0.5
    rho[6, 5, 3] = 0.5
    m[0, 0, 0, 0] = 0.5
    E[0, 0, 0] = 2.75
    m[2, 2, 6, 6] = -0.25
    E[2, 6, 6] = 2.625 + 1.0 / 32
    E[5, 7, 4] = 0.475
    b[1, 1, 2, 1] += 2.0 ** -10
    cfg = mhd.Config(n, n, n, 1.0 / n, gamma=g)
    return dict(rho=rho, m=m, E=E, b=b), cfg


def assert_diag_parity(g, o, U, h):
    """GPU diagnostics ``g`` against the oracle's ``o`` on the same state ``U``:
    totals within 1e-13 of the sum of |x|, min rho and min P within 1e-12
    relative, max|div_h b| within 1e-13 max|b| / h, the unphysical count exact;
    a NaN on one side must be a NaN on the other."""
    import math

    def close(a, b, tol):
        if math.isnan(b) or math.isnan(a):
            return math.isnan(a) and math.isnan(b)
        return abs(a - b) <= tol

    def total_scale(x):
        s = float(x.abs().nansum())
        return s if s > 0 else 1.0

    bad = []
    checks = [("mass", g["mass"], o["mass"], 1e-13 * total_scale(U["rho"])),
              ("energy", g["energy"], o["energy"], 1e-13 * total_scale(U["E"]))]
    for c in range(3):
        checks.append((f"mom{c}", g["mom"][c], o["mom"][c], 1e-13 * total_scale(U["m"][c])))
        checks.append((f"bflux{c}", g["bflux"][c], o["bflux"][c], 1e-13 * total_scale(U["b"][c])))
    checks.append(("min_rho", g["min_rho"], o["min_rho"], 1e-12 * abs(o["min_rho"])))
    checks.append(("min_p", g["min_p"], o["min_p"], 1e-12 * abs(o["min_p"])))
    checks.append(("max_divb", g["max_divb"], o["max_divb"], 1e-13 * float(U["b"].abs().max()) / h))
    for name, a, b, tol in checks:
        if not close(a, b, tol):
            bad.append((name, a, b, tol))
    if g["n_unphysical"] != o["n_unphysical"]:
        bad.append(("n_unphysical", g["n_unphysical"], o["n_unphysical"], 0))
    assert not bad, bad


def walled_state(n=(12, 10, 8), seed=3, v_rms=0.8, walls=(True, False, False)):
    """Generator fields on an nx x ny x nz box whose face field has no normal
    component on the wall faces: the edge potential components tangential to
    each wall vanish on it (edge index n-1 along the walled axis is the wall,
    -1/2 and n-1/2 being the same index), and the uniform field has no normal
    component there; b = B0 + curl_h A keeps div_h b = 0."""
    nx, ny, nz = n
    m = max(n)
    f = inputs.random_fields(m + (m % 2), seed, v_rms, kmax=2, B0=(0.0, 0.0, 0.0))
    rho = np.ascontiguousarray(f.rho[:nz, :ny, :nx])
    v = np.ascontiguousarray(f.v[:, :nz, :ny, :nx])
    A = np.array(f.A[:, :nz, :ny, :nx])
    B0 = [0.3, 0.6, 0.8]
    for axis in range(3):
        if walls[axis]:
            B0[axis] = 0.0
            for c in range(3):
                if c != axis:                       # tangential components on the wall edges
                    idx = [slice(None)] * 3
                    idx[2 - axis] = n[axis] - 1
                    A[(c,) + tuple(idx)] = 0.0
    cfg = mhd.Config(nx, ny, nz, 1.0 / m, walls=tuple(walls))
    U = mhd.init_from_potential(rho, v, A, f.P0, B0, cfg)
    return U, cfg
