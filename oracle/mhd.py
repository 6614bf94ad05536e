"""FP64 CPU oracle: the WENO5-CT ideal-MHD step, written out from the paper.

Test infrastructure (see the package docstring): only the tests, the smoke
check and the CPU-baseline leg of the benchmark use this module.

Layout: scalars on zones are tensors [nz, ny, nx]; grid axis 0 = x is the last
tensor dimension.  A face-centred array ``f`` of direction ``d`` holds at index
(i, j, k) the value on the forward face (i+1/2 along d), the paper's convention
for b (Sect. 2.3).  Edge arrays hold at (i, j, k) the value on the edge that
shares the forward corner: E_z at (i+1/2, j+1/2, k), E_x at (i, j+1/2, k+1/2),
E_y at (i+1/2, j, k+1/2) -- the corner fluxes Omega_x, Omega_y, Omega_z of
eq. (ox1)-(ox3) in that order.

Readings of passages that are garbled or silent:
  R1  total pressure P* = P + |B|^2/2 (eq. for P* drops the parentheses)
  R2  fast/slow speeds c^2 = (a^2 + b^2 +- D)/2 with
      D = sqrt((a^2 - b^2)^2 + 4 a^2 b_perp^2), the expanded radicand of
      eq. (slow)/(fast) with the 1/2 placed on the whole bracket; the slow speed
      from the product of the roots, c_slow^2 = a^2 b_n^2 / c_fast^2
  R3  Alfven speed |B_n|/sqrt(rho)
  R4  Appendix A headings swapped: m = 2, 6 are the Alfven waves, m = 3, 5 slow
  R5  fast-mode left eigenvector: the 1/(2 c_s^2) prefactor applies to every
      component and the components are the ones of the slow row with the
      fast/slow roles exchanged (the printed row is not a left eigenvector)
  R6  entropy right eigenvector energy component v^2/2
  R7  beta normalised by sqrt(B_t1^2 + B_t2^2)
  R8  degenerate branch (alpha_f, alpha_s) = (1/sqrt2, 1/sqrt2); alpha_f^2 and
      alpha_s^2 from (1 +- (a^2 - b^2)/D)/2 clamped to [0, 1], which equals
      eq. (alpha) and is exactly 1/0 when B_perp = 0 (the explicit degeneracy
      setting the appendix recommends); written as (D +- dab)/(2D) with the
      difference D - |dab| formed as 4 a^2 b_perp^2/(D + |dab|), free of the
      cancellation that the appendix's renormalisation near degeneracies guards
  R9  CT transport fluxes T^d_a = F_d[B_a] + <B_d v_a> (the d-face average of
      the two zones), i.e. eq. (fct1)-(fct6) in the frame of each sweep
  R10 face state for L, R: arithmetic mean of the primitive states of the two
      zones sharing the face
  R11 SSP-RK3 (Shu-Osher) in increment form, CFL 0.4, in place of the RK4 of
      Sect. 2.1; classical RK4 is kept as :func:`step_rk4`
  R12 zone-centred B is never advanced by the WENO flux; it is re-interpolated
      from the face field after every stage (Sect. 2.3, 3D step list)
  R13 WENO-Z weights alpha_k = d_k (1 + (tau_5 / (eps_Z + IS_k))^2): the
      printed tau_5 / (eps_Z + IS_k)^2 is dimensionally inconsistent; the
      printed form is kept as weights == 'z_printed'
  R16 the RK4 of Sect. 2.1 as its q_save accumulation (factors 1/2, 1/2, 1,
      1/6 on q0; weights -4/3, 1/3, 2/3, 1/3, 1), dt held over the step
  R20 reflecting walls (the paper's reflecting boundaries, Sect. 4): perfectly
      conducting, ghost zones that mirror the interior (normal momentum and
      normal field odd, everything else even); the corner fluxes on wall edges
      vanish and the normal face field on a wall face is zero
  R21 floors (the protection floors of Sect. 4, unspecified there): after each
      stage, rho below rho_floor is raised to it with the momentum kept, then a
      gas pressure below p_floor is raised to it by adding internal energy;
      activations are counted
"""
from __future__ import annotations

import dataclasses
import math

import torch

DT = torch.float64


@dataclasses.dataclass
class Config:
    nx: int
    ny: int
    nz: int
    h: float                  # zone size (one Delta x for all directions, Sect. 2.3)
    gamma: float = 5.0 / 3.0
    cfl: float = 0.4
    eps: float = 1e-6         # WENO epsilon (Sect. 2.2)
    eps_B: float = 1e-30      # degeneracy threshold (Appendix A)
    weights: str = "js"       # "js" (Jiang-Shu), "z" (WENO-Z) or "z_printed"
    eps_Z: float = 1e-40
    walls: tuple = (False, False, False)   # reflecting conducting walls per axis (R20)
    rho_floor: float = 0.0    # opt-in density floor (R21; 0 = off)
    p_floor: float = 0.0      # opt-in gas-pressure floor (R21; 0 = off)


def cubic(n: int, L: float = 1.0, **kw) -> Config:
    return Config(n, n, n, L / n, **kw)


# ----------------------------------------------------------------------------
# grid helpers
# ----------------------------------------------------------------------------

def at(f: torch.Tensor, o: int, axis: int) -> torch.Tensor:
    """Value at index i+o along grid axis ``axis`` (0=x, 1=y, 2=z), periodic.

    Works for any tensor whose last three dimensions are (z, y, x)."""
    return torch.roll(f, shifts=-o, dims=f.dim() - 1 - axis)


def frame(axis: int):
    """Sweep frame (n, t1, t2): x -> (x, y, z), y -> (y, z, x), z -> (z, x, y)."""
    return axis, (axis + 1) % 3, (axis + 2) % 3


def interp4(b_a: torch.Tensor, axis: int) -> torch.Tensor:
    """Zone-centred component from its face values, fourth order (Sect. 2.3):
    B_i = (-b_{i-2} + 9 b_{i-1} + 9 b_i - b_{i+1}) / 16, b_i on face i+1/2."""
    return (-at(b_a, -2, axis) + 9.0 * at(b_a, -1, axis) + 9.0 * b_a - at(b_a, 1, axis)) / 16.0


def zone_B(b: torch.Tensor) -> torch.Tensor:
    return torch.stack([interp4(b[a], a) for a in range(3)])


def zone_B_cfg(b: torch.Tensor, cfg) -> torch.Tensor:
    """Zone field of a face field with the configuration's walls: along a walled
    axis the fourth-order interpolation reads the mirror ghost faces (R20)."""
    if not any(cfg.walls):
        return zone_B(b)
    D, n = b, [cfg.nx, cfg.ny, cfg.nz]
    for axis in range(3):
        if cfg.walls[axis]:
            D = mirror_double_faces(D, axis)
    B = zone_B(D)
    for axis in range(3):
        if cfg.walls[axis]:
            B = B.narrow(B.dim() - 1 - axis, 0, n[axis])
    return B


def curl_edges(A: torch.Tensor, h: float) -> torch.Tensor:
    """Face field from an edge vector potential by first-order differences
    (Sect. 4.1): b = curl_h A, with A_x at (i, j+1/2, k+1/2) etc."""
    Ax, Ay, Az = A[0], A[1], A[2]
    bx = (Az - at(Az, -1, 1)) / h - (Ay - at(Ay, -1, 2)) / h
    by = (Ax - at(Ax, -1, 2)) / h - (Az - at(Az, -1, 0)) / h
    bz = (Ay - at(Ay, -1, 0)) / h - (Ax - at(Ax, -1, 1)) / h
    return torch.stack([bx, by, bz])


def div_faces(b: torch.Tensor, h: float) -> torch.Tensor:
    """Zone divergence of the face field (the CT constraint, eq. divb)."""
    return ((b[0] - at(b[0], -1, 0)) + (b[1] - at(b[1], -1, 1)) + (b[2] - at(b[2], -1, 2))) / h


# ----------------------------------------------------------------------------
# state
# ----------------------------------------------------------------------------

def init_from_potential(rho, v, A, P0: float, B0, cfg: Config):
    """Conserved state from primitive fields and an edge vector potential:
    b = B0 + curl_h A, zone B by fourth-order interpolation, m = rho v and
    E = P/(gamma-1) + (rho v^2 + B^2)/2 (eq. P).  With walls (R20) the normal
    field on the wall faces is set to zero."""
    rho = torch.as_tensor(rho, dtype=DT)
    v = torch.as_tensor(v, dtype=DT)
    A = torch.as_tensor(A, dtype=DT)
    b = curl_edges(A, cfg.h)
    b = torch.stack([b[a] + float(B0[a]) for a in range(3)])
    for axis in range(3):                       # a wall face carries no normal field (R20)
        if cfg.walls[axis]:
            b[axis].narrow(b[axis].dim() - 1 - axis, b[axis].shape[-1 - axis] - 1, 1).zero_()
    B = zone_B_cfg(b, cfg)
    m = rho * v
    E = P0 / (cfg.gamma - 1.0) + 0.5 * (rho * (v * v).sum(0) + (B * B).sum(0))
    return dict(rho=rho, m=m, E=E, b=b)


def primitives(U, gamma: float, cfg=None):
    """rho, v, zone B and gas pressure from the conserved state (eq. P); with a
    configuration, zone B follows its walls."""
    rho, m, E = U["rho"], U["m"], U["E"]
    B = zone_B(U["b"]) if cfg is None else zone_B_cfg(U["b"], cfg)
    v = m / rho
    P = (gamma - 1.0) * (E - 0.5 * ((m * v).sum(0) + (B * B).sum(0)))
    return rho, v, B, P


# ----------------------------------------------------------------------------
# fluxes, wave speeds, eigensystem (Sect. 2, Appendix A), in a sweep frame
# ----------------------------------------------------------------------------

def flux_vector(rho, mn, mt1, mt2, E, vn, vt1, vt2, Bn, Bt1, Bt2, P):
    """The seven non-trivial components of the flux along n, eq. (fluxes), in the
    order of the characteristic state (rho, m_n, m_t1, m_t2, B_t1, B_t2, E).
    The B_n component is identically zero and B_n is a parameter."""
    Pstar = P + 0.5 * (Bn * Bn + Bt1 * Bt1 + Bt2 * Bt2)              # R1
    vB = vn * Bn + vt1 * Bt1 + vt2 * Bt2
    return torch.stack([
        rho * vn,
        rho * vn * vn + Pstar - Bn * Bn,
        rho * vn * vt1 - Bn * Bt1,
        rho * vn * vt2 - Bn * Bt2,
        Bt1 * vn - Bn * vt1,
        Bt2 * vn - Bn * vt2,
        (E + Pstar) * vn - Bn * vB,
    ], dim=-1)


def wave_speeds(rho, Bn, Bt1, Bt2, P, gamma: float):
    """c_fast, c_A, c_slow along n, eq. (slow), (fast), (ca) with readings R2, R3."""
    a2 = gamma * P / rho                     # c_s^2
    b2 = (Bn * Bn + Bt1 * Bt1 + Bt2 * Bt2) / rho
    bn2 = Bn * Bn / rho
    bperp2 = (Bt1 * Bt1 + Bt2 * Bt2) / rho
    D = torch.sqrt((a2 - b2) ** 2 + 4.0 * a2 * bperp2)
    cf2 = 0.5 * (a2 + b2 + D)
    cs2 = torch.where(cf2 > 0, a2 * bn2 / torch.where(cf2 > 0, cf2, torch.ones_like(cf2)),
                      torch.zeros_like(cf2))
    return torch.sqrt(cf2), torch.sqrt(bn2), torch.sqrt(cs2)


def eigenvalues(vn, c_fast, c_A, c_slow):
    """lambda(m), m = 1..7: v -+ c_fast, v -+ c_A, v -+ c_slow, v (Appendix A)."""
    return torch.stack([vn - c_fast, vn - c_A, vn - c_slow, vn,
                        vn + c_slow, vn + c_A, vn + c_fast], dim=-1)


def eigenvectors(rho, vn, vt1, vt2, Bn, Bt1, Bt2, P, gamma: float, eps_B: float):
    """Left and right eigenvectors of the 7x7 flux Jacobian (Appendix A).

    Returns L[..., m, j] (row m is L(m)) and R[..., j, m] (column m is R(m)),
    with the upper signs of the appendix for m = 1, 2, 3 (lambda = v - c) and
    the lower signs for m = 7, 6, 5.  Readings R2, R4-R8 apply."""
    a2 = gamma * P / rho
    cs = torch.sqrt(a2)                                   # sound speed, stored (Appendix A)
    sr = torch.sqrt(rho)
    b2 = (Bn * Bn + Bt1 * Bt1 + Bt2 * Bt2) / rho
    Bperp2 = Bt1 * Bt1 + Bt2 * Bt2
    D = torch.sqrt((a2 - b2) ** 2 + 4.0 * a2 * Bperp2 / rho)
    cf2 = 0.5 * (a2 + b2 + D)
    c_fast = torch.sqrt(cf2)
    cs2_slow = torch.where(cf2 > 0, a2 * (Bn * Bn / rho) / torch.where(cf2 > 0, cf2, torch.ones_like(cf2)),
                           torch.zeros_like(cf2))
    c_slow = torch.sqrt(cs2_slow)

    # beta (R7) and sgn(B_n)
    big = Bperp2 > eps_B
    nb = torch.sqrt(torch.where(big, Bperp2, torch.ones_like(Bperp2)))
    beta_y = torch.where(big, Bt1 / nb, torch.full_like(Bt1, 1.0 / math.sqrt(2.0)))
    beta_z = torch.where(big, Bt2 / nb, torch.full_like(Bt2, 1.0 / math.sqrt(2.0)))
    sgn = torch.where(Bn >= eps_B, torch.ones_like(Bn), -torch.ones_like(Bn))

    # alpha_f, alpha_s (eq. alpha, R8): alpha_f^2 = (1 + r)/2 = (D + dab)/(2D),
    # alpha_s^2 = (1 - r)/2 = (D - dab)/(2D), with D - |dab| = 4 a^2 b_perp^2 / (D + |dab|)
    # (D^2 = dab^2 + 4 a^2 b_perp^2), so the smaller one carries no cancellation
    nondeg = torch.sqrt(D) >= eps_B
    Dsafe = torch.where(nondeg, D, torch.ones_like(D))
    dab = a2 - b2
    big = (Dsafe + dab.abs()) / (2.0 * Dsafe)
    small = 4.0 * a2 * Bperp2 / rho / (Dsafe + dab.abs()) / (2.0 * Dsafe)
    af2 = torch.clamp(torch.where(dab >= 0, big, small), 0.0, 1.0)
    as2 = torch.clamp(torch.where(dab >= 0, small, big), 0.0, 1.0)
    alpha_f = torch.where(nondeg, torch.sqrt(af2), torch.full_like(D, 1.0 / math.sqrt(2.0)))
    alpha_s = torch.where(nondeg, torch.sqrt(as2), torch.full_like(D, 1.0 / math.sqrt(2.0)))

    gamma_1 = (gamma - 1.0) / 2.0
    gamma_2 = (gamma - 2.0) / (gamma - 1.0)
    tau = (gamma - 1.0) / a2
    v2 = vn * vn + vt1 * vt1 + vt2 * vt2
    bv = beta_y * vt1 + beta_z * vt2
    Gamma_f = alpha_f * c_fast * vn - alpha_s * c_slow * sgn * bv
    Gamma_a = sgn * (beta_z * vt1 - beta_y * vt2)
    Gamma_s = alpha_s * c_slow * vn + alpha_f * c_fast * sgn * bv
    half_a2 = 1.0 / (2.0 * a2)
    zero = torch.zeros_like(rho)
    one = torch.ones_like(rho)

    L_rows = [None] * 7
    R_cols = [None] * 7
    for m, sg in ((0, +1.0), (6, -1.0)):        # fast: m=1 upper (+), m=7 lower (-)
        L_rows[m] = [half_a2 * (alpha_f * gamma_1 * v2 + sg * Gamma_f),
                     half_a2 * ((1.0 - gamma) * alpha_f * vn - sg * alpha_f * c_fast),
                     half_a2 * ((1.0 - gamma) * alpha_f * vt1 + sg * c_slow * alpha_s * beta_y * sgn),
                     half_a2 * ((1.0 - gamma) * alpha_f * vt2 + sg * c_slow * alpha_s * beta_z * sgn),
                     half_a2 * ((1.0 - gamma) * alpha_f * Bt1 + sr * cs * alpha_s * beta_y),
                     half_a2 * ((1.0 - gamma) * alpha_f * Bt2 + sr * cs * alpha_s * beta_z),
                     half_a2 * ((gamma - 1.0) * alpha_f)]
        R_cols[m] = [alpha_f,
                     alpha_f * (vn - sg * c_fast),
                     alpha_f * vt1 + sg * c_slow * alpha_s * beta_y * sgn,
                     alpha_f * vt2 + sg * c_slow * alpha_s * beta_z * sgn,
                     cs * alpha_s * beta_y / sr,
                     cs * alpha_s * beta_z / sr,
                     alpha_f * (0.5 * v2 + c_fast * c_fast - gamma_2 * a2) - sg * Gamma_f]
    for m, sg in ((1, +1.0), (5, -1.0)):        # Alfven (R4): m=2 upper, m=6 lower
        L_rows[m] = [0.5 * Gamma_a, zero,
                     -0.5 * beta_z * sgn, 0.5 * beta_y * sgn,
                     -sg * 0.5 * sr * beta_z, sg * 0.5 * sr * beta_y, zero]
        R_cols[m] = [zero, zero,
                     -beta_z * sgn, beta_y * sgn,
                     -sg * beta_z / sr, sg * beta_y / sr, -Gamma_a]
    for m, sg in ((2, +1.0), (4, -1.0)):        # slow (R4): m=3 upper, m=5 lower
        L_rows[m] = [half_a2 * (gamma_1 * alpha_s * v2 + sg * Gamma_s),
                     half_a2 * ((1.0 - gamma) * alpha_s * vn - sg * alpha_s * c_slow),
                     half_a2 * ((1.0 - gamma) * alpha_s * vt1 - sg * c_fast * alpha_f * beta_y * sgn),
                     half_a2 * ((1.0 - gamma) * alpha_s * vt2 - sg * c_fast * alpha_f * beta_z * sgn),
                     half_a2 * ((1.0 - gamma) * alpha_s * Bt1 - sr * cs * alpha_f * beta_y),
                     half_a2 * ((1.0 - gamma) * alpha_s * Bt2 - sr * cs * alpha_f * beta_z),
                     half_a2 * ((gamma - 1.0) * alpha_s)]
        R_cols[m] = [alpha_s,
                     alpha_s * (vn - sg * c_slow),
                     alpha_s * vt1 - sg * c_fast * alpha_f * beta_y * sgn,
                     alpha_s * vt2 - sg * c_fast * alpha_f * beta_z * sgn,
                     -cs * alpha_f * beta_y / sr,
                     -cs * alpha_f * beta_z / sr,
                     alpha_s * (0.5 * v2 + c_slow * c_slow - gamma_2 * a2) - sg * Gamma_s]
    L_rows[3] = [1.0 - 0.5 * tau * v2, tau * vn, tau * vt1, tau * vt2, tau * Bt1, tau * Bt2, -tau * one]
    R_cols[3] = [one, vn, vt1, vt2, zero, zero, 0.5 * v2]                       # R6

    L = torch.stack([torch.stack(row, dim=-1) for row in L_rows], dim=-2)      # [..., m, j]
    R = torch.stack([torch.stack(col, dim=-1) for col in R_cols], dim=-1)      # [..., j, m]
    return L, R


# ----------------------------------------------------------------------------
# WENO5 (Sect. 2.2)
# ----------------------------------------------------------------------------

def phi_N(a, b, c, d, cfg: Config):
    """The WENO interpolant phi_N(a, b, c, d) of eq. (FWENO) with the Jiang-Shu
    weights (or the WENO-Z weights of reading R13 when cfg.weights == 'z', or
    the WENO-Z weights exactly as Sect. 2.2 prints them when 'z_printed')."""
    IS_0 = 13.0 * (a - b) ** 2 + 3.0 * (a - 3.0 * b) ** 2
    IS_1 = 13.0 * (b - c) ** 2 + 3.0 * (b + c) ** 2
    IS_2 = 13.0 * (c - d) ** 2 + 3.0 * (3.0 * c - d) ** 2
    if cfg.weights == "js":
        alpha_0 = 1.0 / (cfg.eps + IS_0) ** 2
        alpha_1 = 6.0 / (cfg.eps + IS_1) ** 2
        alpha_2 = 3.0 / (cfg.eps + IS_2) ** 2
    elif cfg.weights == "z":
        tau_5 = torch.abs(IS_0 - IS_2)
        alpha_0 = 1.0 * (1.0 + (tau_5 / (cfg.eps_Z + IS_0)) ** 2)
        alpha_1 = 6.0 * (1.0 + (tau_5 / (cfg.eps_Z + IS_1)) ** 2)
        alpha_2 = 3.0 * (1.0 + (tau_5 / (cfg.eps_Z + IS_2)) ** 2)
    elif cfg.weights == "z_printed":
        tau_5 = torch.abs(IS_0 - IS_2)
        alpha_0 = 1.0 * (1.0 + tau_5 / (cfg.eps_Z + IS_0) ** 2)
        alpha_1 = 6.0 * (1.0 + tau_5 / (cfg.eps_Z + IS_1) ** 2)
        alpha_2 = 3.0 * (1.0 + tau_5 / (cfg.eps_Z + IS_2) ** 2)
    else:
        raise ValueError(cfg.weights)
    s = alpha_0 + alpha_1 + alpha_2
    omega_0 = alpha_0 / s
    omega_2 = alpha_2 / s
    return omega_0 * (a - 2.0 * b + c) / 3.0 + (omega_2 - 0.5) * (b - 2.0 * c + d) / 6.0


def weno_split_flux(Fs, qs, alpha, cfg: Config):
    """Characteristic flux at i+1/2 from projected zone values, eq. (FWENO).

    ``Fs[k]``, ``qs[k]`` for k = 0..5 are F^s, q^s of zones i-2 .. i+3 (any
    trailing shape); ``alpha`` the Lax-Friedrichs speed of each component."""
    dF = [Fs[k + 1] - Fs[k] for k in range(5)]       # Delta F^s at i-3/2 .. i+5/2
    dq = [qs[k + 1] - qs[k] for k in range(5)]
    dFp = [0.5 * (dF[k] + alpha * dq[k]) for k in range(5)]
    dFm = [0.5 * (dF[k] - alpha * dq[k]) for k in range(5)]
    central = (-Fs[1] + 7.0 * Fs[2] + 7.0 * Fs[3] - Fs[4]) / 12.0
    return (central
            - phi_N(dFp[0], dFp[1], dFp[2], dFp[3], cfg)
            + phi_N(dFm[4], dFm[3], dFm[2], dFm[1], cfg))


def lf_speed(lam, axis: int):
    """alpha(m) = max(|lambda_i(m)|, |lambda_{i+1}(m)|) on face i+1/2 (Sect. 2.2),
    for zone eigenvalues ``lam`` [..., 7]."""
    return torch.maximum(lam.abs(), at(lam.movedim(-1, 0), 1, axis).movedim(0, -1).abs())


# ----------------------------------------------------------------------------
# one directional sweep
# ----------------------------------------------------------------------------

def sweep(U, axis: int, cfg: Config, prims=None):
    """WENO fluxes on the forward faces along ``axis`` (Sect. 2.2, 3D step list).

    Returns (F_face, T): F_face[..., 7] the interface flux in the sweep frame,
    T[2, ...] the CT transport fluxes T^n_t1, T^n_t2 of eq. (fct1)-(fct6) (R9)."""
    rho, v, B, P = prims if prims is not None else primitives(U, cfg.gamma)
    n, t1, t2 = frame(axis)
    m, E = U["m"], U["E"]
    vn, vt1, vt2 = v[n], v[t1], v[t2]
    Bn, Bt1, Bt2 = B[n], B[t1], B[t2]

    # zone values (steps 2 of the 3D step list): state q, flux F, eigenvalues
    q = torch.stack([rho, m[n], m[t1], m[t2], Bt1, Bt2, E], dim=-1)
    F = flux_vector(rho, m[n], m[t1], m[t2], E, vn, vt1, vt2, Bn, Bt1, Bt2, P)
    c_fast, c_A, c_slow = wave_speeds(rho, Bn, Bt1, Bt2, P, cfg.gamma)
    lam = eigenvalues(vn, c_fast, c_A, c_slow)

    # face state by arithmetic averaging of zones i and i+1 (R10)
    def face(x):
        return 0.5 * (x + at(x, 1, axis))
    L, R = eigenvectors(face(rho), face(vn), face(vt1), face(vt2), face(Bn), face(Bt1),
                        face(Bt2), face(P), cfg.gamma, cfg.eps_B)
    alpha = lf_speed(lam, axis)

    # characteristic projections F^s_k(m) = L(m).F_k, q^s_k(m) = L(m).q_k, k = i-2..i+3
    def shifted(x, o):
        return at(x.movedim(-1, 0), o, axis).movedim(0, -1)
    Fs = [torch.einsum("...mj,...j->...m", L, shifted(F, o)) for o in range(-2, 4)]
    qs = [torch.einsum("...mj,...j->...m", L, shifted(q, o)) for o in range(-2, 4)]
    Fs_face = weno_split_flux(Fs, qs, alpha, cfg)
    F_face = torch.einsum("...jm,...m->...j", R, Fs_face)

    # CT transport fluxes (R9): the B_t components plus the face mean of B_n v_t
    T = torch.stack([F_face[..., 4] + face(Bn * vt1), F_face[..., 5] + face(Bn * vt2)])
    return F_face, T


# ----------------------------------------------------------------------------
# right-hand side, CT, time step
# ----------------------------------------------------------------------------

def rhs(U, cfg: Config, return_parts: bool = False):
    """dU/dt of the semi-discrete scheme (periodic, or with the walls of
    cfg.walls: :func:`rhs_walled`)."""
    if any(cfg.walls):
        if return_parts:
            raise ValueError("parts are for the periodic scheme")
        return rhs_walled(U, cfg)
    return rhs_periodic(U, cfg, return_parts)


def rhs_periodic(U, cfg: Config, return_parts: bool = False):
    """dU/dt of the semi-discrete scheme: conservative WENO flux divergence
    (eq. num) for rho, m, E summed over the three sweeps, and the CT update of
    the face field from the corner fluxes (eq. ox1-ox3 and the b equations)."""
    h = cfg.h
    prims = primitives(U, cfg.gamma)
    k_rho = torch.zeros_like(U["rho"])
    k_m = torch.zeros_like(U["m"])
    k_E = torch.zeros_like(U["E"])
    Tt = {}
    parts = {}
    for axis in range(3):
        n, t1, t2 = frame(axis)
        F_face, T = sweep(U, axis, cfg, prims)
        div = [-(F_face[..., c] - at(F_face[..., c], -1, axis)) / h for c in range(7)]
        k_rho = k_rho + div[0]
        k_m = k_m + torch.stack([div[1 + [n, t1, t2].index(c)] for c in range(3)])
        k_E = k_E + div[6]
        Tt[(axis, t1)] = T[0]
        Tt[(axis, t2)] = T[1]
        parts[axis] = (F_face, T)
    X, Y, Z = 0, 1, 2
    f_y, f_z = Tt[(X, Y)], Tt[(X, Z)]       # f*_y, f*_z on x-faces
    g_z, g_x = Tt[(Y, Z)], Tt[(Y, X)]       # g*_z, g*_x on y-faces
    h_x, h_y = Tt[(Z, X)], Tt[(Z, Y)]       # h*_x, h*_y on z-faces
    Omega_x = 0.5 * (g_x + at(g_x, 1, X)) - 0.5 * (f_y + at(f_y, 1, Y))   # eq. (ox1), edge (i+1/2, j+1/2, k)
    Omega_y = 0.5 * (h_y + at(h_y, 1, Y)) - 0.5 * (g_z + at(g_z, 1, Z))   # eq. (ox2), edge (i, j+1/2, k+1/2)
    Omega_z = 0.5 * (f_z + at(f_z, 1, Z)) - 0.5 * (h_x + at(h_x, 1, X))   # eq. (ox3), edge (i+1/2, j, k+1/2)
    k = dict(rho=k_rho, m=k_m, E=k_E, b=face_field_rhs(Omega_x, Omega_y, Omega_z, h))
    if return_parts:
        return k, dict(sweeps=parts, Omega=(Omega_x, Omega_y, Omega_z))
    return k


def face_field_rhs(Omega_x, Omega_y, Omega_z, h: float):
    """db/dt = -curl_h of the corner fluxes (the b equations of Sect. 2.3):
    Omega_x = E_z at (i+1/2, j+1/2, k), Omega_y = E_x at (i, j+1/2, k+1/2),
    Omega_z = E_y at (i+1/2, j, k+1/2)."""
    X, Y, Z = 0, 1, 2
    k_bx = -(Omega_x - at(Omega_x, -1, Y)) / h + (Omega_z - at(Omega_z, -1, Z)) / h
    k_by = -(Omega_y - at(Omega_y, -1, Z)) / h + (Omega_x - at(Omega_x, -1, X)) / h
    k_bz = -(Omega_z - at(Omega_z, -1, X)) / h + (Omega_y - at(Omega_y, -1, Y)) / h
    return torch.stack([k_bx, k_by, k_bz])


# ----------------------------------------------------------------------------
# reflecting walls (R20) and floors (R21)
# ----------------------------------------------------------------------------

def _zone_dim(t: torch.Tensor, axis: int) -> int:
    return t.dim() - 1 - axis


def mirror_double(U, axis: int):
    """The state extended to 2N zones along ``axis`` by its mirror image about
    the upper wall face (N-1/2): zone N+m is zone N-1-m with the normal momentum
    negated; the normal face field is odd about both wall faces (N-1/2 and
    -1/2 = 2N-1/2, where it is zero), the tangential face fields even.  These are
    the ghost zones of a reflecting, perfectly conducting wall."""
    def ext(f, sign=1.0):
        d = _zone_dim(f, axis)
        return torch.cat([f, sign * torch.flip(f, dims=[d])], dim=d)
    m = torch.stack([ext(U["m"][c], -1.0 if c == axis else 1.0) for c in range(3)])
    return dict(rho=ext(U["rho"]), m=m, E=ext(U["E"]), b=mirror_double_faces(U["b"], axis))


def mirror_double_faces(b: torch.Tensor, axis: int) -> torch.Tensor:
    """The face field part of :func:`mirror_double`."""
    bs = []
    for c in range(3):
        f = b[c]
        d = _zone_dim(f, axis)
        if c != axis:
            bs.append(torch.cat([f, torch.flip(f, dims=[d])], dim=d))
            continue
        n = f.shape[d]
        # doubled faces N..2N-2 are -b(N-2..0); face 2N-1 is the lower wall
        tail = -torch.flip(f.narrow(d, 0, n - 1), dims=[d])
        bs.append(torch.cat([f, tail, torch.zeros_like(f.narrow(d, 0, 1))], dim=d))
    return torch.stack(bs)


def rhs_walled(U, cfg: Config):
    """Right-hand side with reflecting conducting walls on the axes cfg.walls
    marks (R20): the periodic scheme on the box mirror-doubled along each
    walled axis (ghost zones that mirror the interior), restricted to the
    original zones, with the corner fluxes on the wall edges set to zero (the
    tangential electric field of a conducting wall) and the normal face field
    on the wall faces held at zero."""
    D = U
    sizes = [cfg.nx, cfg.ny, cfg.nz]
    for axis in range(3):
        if cfg.walls[axis]:
            D = mirror_double(D, axis)
            sizes[axis] *= 2
    cfgD = dataclasses.replace(cfg, nx=sizes[0], ny=sizes[1], nz=sizes[2], walls=(False, False, False))
    k, parts = rhs_periodic(D, cfgD, return_parts=True)
    Ox, Oy, Oz = [o.clone() for o in parts["Omega"]]
    n = [cfg.nx, cfg.ny, cfg.nz]
    # wall planes of the doubled box along a walled axis: faces N-1 and 2N-1
    for axis in range(3):
        if not cfg.walls[axis]:
            continue
        for o, on_axis in ((Ox, (0, 1)), (Oy, (1, 2)), (Oz, (0, 2))):
            if axis in on_axis:            # the edge lies in planes of constant axis
                d = _zone_dim(o, axis)
                o.index_fill_(d, torch.tensor([n[axis] - 1, 2 * n[axis] - 1]), 0.0)
    kb = face_field_rhs(Ox, Oy, Oz, cfg.h)

    def crop(f):
        for axis in range(3):
            if cfg.walls[axis]:
                f = f.narrow(_zone_dim(f, axis), 0, n[axis])
        return f
    out = dict(rho=crop(k["rho"]), m=crop(k["m"]), E=crop(k["E"]), b=crop(kb))
    for axis in range(3):
        if cfg.walls[axis]:
            out["b"][axis].narrow(_zone_dim(out["b"][axis], axis), n[axis] - 1, 1).zero_()
    return out


def apply_floors(U, cfg: Config):
    """Opt-in floors (R21) on a stage result: rho < rho_floor is raised to the
    floor (momentum kept), then a gas pressure below p_floor (eq. P with the
    zone field of the state's face field) is raised to the floor by adding
    internal energy.  Returns (state, number of activations)."""
    n = 0
    rho, m, E = U["rho"], U["m"], U["E"]
    if cfg.rho_floor > 0:
        low = rho < cfg.rho_floor
        n += int(low.sum())
        rho = torch.where(low, torch.full_like(rho, cfg.rho_floor), rho)
    if cfg.p_floor > 0:
        _, _, _, P = primitives(dict(rho=rho, m=m, E=E, b=U["b"]), cfg.gamma, cfg)
        low = P < cfg.p_floor
        n += int(low.sum())
        E = torch.where(low, E + (cfg.p_floor - P) / (cfg.gamma - 1.0), E)
    return dict(rho=rho, m=m, E=E, b=U["b"]), n


def max_signal_speeds(U, cfg: Config):
    """max over zones of |v_d| + c_fast^d for d = x, y, z (denominator of eq. cfl)."""
    rho, v, B, P = primitives(U, cfg.gamma, cfg)
    out = []
    for axis in range(3):
        n, t1, t2 = frame(axis)
        c_fast, _, _ = wave_speeds(rho, B[n], B[t1], B[t2], P, cfg.gamma)
        out.append(torch.max(v[n].abs() + c_fast))
    return torch.stack(out)


def compute_dt(U, cfg: Config) -> float:
    """Time step of eq. (cfl), taken at equality with cfg.cfl."""
    s = max_signal_speeds(U, cfg)
    return float(cfg.cfl * cfg.h / s.sum())


def _axpy(U, k, c):
    return {key: U[key] + c * k[key] for key in U}


def rk_stage(stage: int, Un, acc, Us, dt: float, cfg: Config):
    """One SSP-RK3 stage in increment form (R11).

    stage 0: acc = k0,        U1 = Un + dt acc
    stage 1: acc = k0 + k1,   U2 = Un + dt/4 acc
    stage 2:                  Un+1 = Un + dt/6 (acc + 4 k2)
    Returns (acc, U_next)."""
    k = rhs(Us, cfg)
    if stage == 0:
        acc = {key: k[key] for key in k}
        return acc, _axpy(Un, acc, dt)
    if stage == 1:
        acc = {key: acc[key] + k[key] for key in k}
        return acc, _axpy(Un, acc, 0.25 * dt)
    if stage == 2:
        tot = {key: acc[key] + 4.0 * k[key] for key in k}
        return acc, _axpy(Un, tot, dt / 6.0)
    raise ValueError(stage)


def step(U, cfg: Config, dt: float | None = None, stats: dict | None = None):
    """One SSP-RK3 step; dt from eq. (cfl) on U unless given.  Returns (U, dt).
    With floors (R21) each stage result is floored; the activations are added
    to stats["n_floored"] when a dict is given."""
    if dt is None:
        dt = compute_dt(U, cfg)
    floors = cfg.rho_floor > 0 or cfg.p_floor > 0

    def fl(V):
        if not floors:
            return V
        V, n = apply_floors(V, cfg)
        if stats is not None:
            stats["n_floored"] = stats.get("n_floored", 0) + n
        return V
    acc, U1 = rk_stage(0, U, None, U, dt, cfg)
    U1 = fl(U1)
    acc, U2 = rk_stage(1, U, acc, U1, dt, cfg)
    U2 = fl(U2)
    _, U3 = rk_stage(2, U, acc, U2, dt, cfg)
    return fl(U3), dt


def step_rk4(U, cfg: Config, dt: float | None = None):
    """The classical four-stage RK4 of Sect. 2.1 with the q_save accumulator."""
    if dt is None:
        dt = compute_dt(U, cfg)
    q0 = U
    q_save = {key: -4.0 / 3.0 * q0[key] for key in q0}
    q = q0
    for fac, w in ((0.5, 1.0 / 3.0), (0.5, 2.0 / 3.0), (1.0, 1.0 / 3.0), (1.0 / 6.0, 1.0)):
        k = rhs(q, cfg)
        q = _axpy(q0, k, fac * dt)
        q_save = {key: q_save[key] + w * q[key] for key in q}
    return q_save, dt


# ----------------------------------------------------------------------------
# diagnostics
# ----------------------------------------------------------------------------

def diagnostics(U, cfg: Config):
    """max|div_h b| (eq. divb; NaN if any divergence is NaN), totals of rho, m,
    E, face-b sums, min rho and min P over the zones where they are not NaN
    (NaN zones are reported by the count instead), and the number of zones with
    rho <= 0, P <= 0 or a non-finite rho, P or E."""
    rho, v, B, P = primitives(U, cfg.gamma, cfg)
    bad = (rho <= 0) | (P <= 0) | ~torch.isfinite(rho) | ~torch.isfinite(P) | ~torch.isfinite(U["E"])

    def nanmin(x):
        x = x[~torch.isnan(x)]
        return float(x.min()) if x.numel() else math.inf

    return dict(
        max_divb=float(div_faces(U["b"], cfg.h).abs().max()),
        mass=float(U["rho"].sum()),
        mom=[float(U["m"][c].sum()) for c in range(3)],
        energy=float(U["E"].sum()),
        bflux=[float(U["b"][c].sum()) for c in range(3)],
        min_rho=nanmin(rho),
        min_p=nanmin(P),
        n_unphysical=int(bad.sum()),
    )


def wave_rms(U, e, background: float) -> float:
    """Root-mean-square fluctuation of the zone field's component along the unit
    vector e (a wave-frame axis) about its background value, over all zones:
    the delta B_y of eq. (decay_rate) for e = the wave frame's second axis."""
    B = zone_B(U["b"])
    comp = B[0] * float(e[0]) + B[1] * float(e[1]) + B[2] * float(e[2])
    return float(((comp - background) ** 2).mean().sqrt())


def decay_rate(rms_0: float, rms_t: float, t: float) -> float:
    """Eq. (decay_rate): tau_D = -log(delta B_y(t) / delta B_y(0)) / t."""
    return -math.log(rms_t / rms_0) / t


def l1_error(Ua, Ub, n_zones: int | None = None):
    """Per-variable L1 and the geometric norm of Sect. 3 (eq. for L_1).

    Variables: rho, m_x, m_y, m_z, zone B_x, B_y, B_z, E."""
    def comps(U):
        B = zone_B(U["b"])
        return [U["rho"], U["m"][0], U["m"][1], U["m"][2], B[0], B[1], B[2], U["E"]]
    ca, cb = comps(Ua), comps(Ub)
    N = n_zones or ca[0].numel()
    per = [float((x - y).abs().sum() / N) for x, y in zip(ca, cb)]
    return per, math.sqrt(sum(p * p for p in per))
