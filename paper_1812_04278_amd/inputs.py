"""Seeded synthetic input fields for the WENO5-CT MHD step.

This module draws random Fourier coefficients and evaluates them on the
staggered mesh.  It holds none of the method's arithmetic: no curl, no
interpolation, no energy or flux.  It returns the raw initial fields that both
the HIP path and the CPU oracle turn into a conserved state on their own:

* ``rho``   zone-centred density                      [nz, ny, nx]
* ``v``     zone-centred velocity (x, y, z)           [3, nz, ny, nx]
* ``A``     edge-centred vector potential (x, y, z)   [3, nz, ny, nx]
            A_x at (i, j+1/2, k+1/2), A_y at (i+1/2, j, k+1/2),
            A_z at (i+1/2, j+1/2, k), the placement of Sect. 4.1 (linear waves)
* ``B0``, ``P0`` uniform background field and pressure.

Recipe:

* mode set K(kmax) = {k in Z^3 : 0 < |k| <= kmax}, one representative of each
  +-k pair (k_z > 0, or k_z = 0 and k_y > 0, or k_z = k_y = 0 and k_x > 0),
  listed in lexicographic (k_z, k_y, k_x) order;
* density  rho = 1 + 0.1 * sum_{n<8} sin(2 pi k_n . x + phi_n), k_n uniform
  in K(min(kmax, 4)), phi_n uniform in [0, 2 pi);
* velocity v = sum_{k in K} a_k cos(2 pi k.x) + c_k sin(2 pi k.x), a_k, c_k
  standard normal 3-vectors, scaled so that the grid rms of |v| is ``v_rms``;
* potential A: same form with its own draws, scaled so that the rms of the
  continuous field curl A is ``b_rms``;
* the box is the unit cube, zone centres at ((i+1/2)h, (j+1/2)h, (k+1/2)h).

Draw order from ``numpy.random.Generator(PCG64(seed))``: the 8 density mode
indices, the 8 density phases, then a_k, c_k for every velocity mode (each a
3-vector, in mode order), then the same for A.  The Fourier sums are evaluated
with an inverse FFT on the N^3 grid (exact for N > 2 kmax), so the same seed
sampled at a smaller N gives the same continuous field.
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = ["Fields", "mode_set", "random_fields", "config_fields", "fast_wave"]


@dataclasses.dataclass
class Fields:
    rho: np.ndarray          # [nz, ny, nx] float64
    v: np.ndarray            # [3, nz, ny, nx] float64
    A: np.ndarray            # [3, nz, ny, nx] float64 (edge placement above)
    B0: tuple                # uniform field (Bx, By, Bz)
    P0: float                # uniform pressure
    gamma: float = 5.0 / 3.0


def mode_set(kmax: int) -> np.ndarray:
    """Half-space representatives of the integer wave vectors with 0<|k|<=kmax."""
    out = []
    r = int(kmax)
    for kz in range(-r, r + 1):
        for ky in range(-r, r + 1):
            for kx in range(-r, r + 1):
                k2 = kx * kx + ky * ky + kz * kz
                if k2 == 0 or k2 > kmax * kmax:
                    continue
                if kz > 0 or (kz == 0 and ky > 0) or (kz == 0 and ky == 0 and kx > 0):
                    out.append((kx, ky, kz))
    return np.array(out, dtype=np.int64)


def _evaluate(n: int, ks: np.ndarray, a: np.ndarray, c: np.ndarray, offset) -> np.ndarray:
    """sum_k a_k cos(2 pi k.x) + c_k sin(2 pi k.x) at x = (idx + offset)/n.

    ``offset`` is (ox, oy, oz) in units of the zone size.  Returns [nz, ny, nx].
    """
    if 2 * int(np.abs(ks).max()) >= n:
        raise ValueError(f"grid n={n} too small for modes up to |k_i|={np.abs(ks).max()}")
    grid = np.zeros((n, n, n), dtype=np.complex128)
    ox, oy, oz = offset
    for (kx, ky, kz), ak, ck in zip(ks, a, c):
        phase = np.exp(2j * np.pi * (kx * ox + ky * oy + kz * oz) / n)
        coef = (ak - 1j * ck) * phase            # a cos + c sin = Re[(a - i c) e^{i theta}]
        grid[kz % n, ky % n, kx % n] += coef
    # f[idx] = Re sum_k C_k exp(2 pi i k.idx / n) = Re(n^3 * ifftn(grid))
    return np.real(np.fft.ifftn(grid) * (n ** 3))


def _evaluate_device(n: int, ks: np.ndarray, a: np.ndarray, c: np.ndarray, offset, device):
    """:func:`_evaluate` with the inverse FFT on a torch device (same sums, another
    FFT: the values agree to rounding).  Returns a float64 tensor [nz, ny, nx]."""
    import torch
    if 2 * int(np.abs(ks).max()) >= n:
        raise ValueError(f"grid n={n} too small for modes up to |k_i|={np.abs(ks).max()}")
    ox, oy, oz = offset
    phase = np.exp(2j * np.pi * (ks[:, 0] * ox + ks[:, 1] * oy + ks[:, 2] * oz) / n)
    coef = torch.as_tensor((a - 1j * c) * phase, dtype=torch.complex128, device=device)
    idx = torch.as_tensor(((ks[:, 2] % n) * n + (ks[:, 1] % n)) * n + (ks[:, 0] % n), device=device)
    grid = torch.zeros(n * n * n, dtype=torch.complex128, device=device)
    grid.index_add_(0, idx, coef)
    out = torch.fft.ifftn(grid.view(n, n, n)).real * float(n ** 3)
    del grid
    return out.contiguous()


# positions of the velocity (zone centres) and of the potential components
# (edges) in units of the zone size
V_OFFSET = (0.5, 0.5, 0.5)
EDGE_OFFSETS = [(0.5, 1.0, 1.0), (1.0, 0.5, 1.0), (1.0, 1.0, 0.5)]


def fourier_modes(seed: int, v_rms: float, kmax: int = 4, b_rms: float = 0.1) -> dict:
    """The draws of :func:`random_fields` and the Fourier amplitudes it evaluates:
    ``kset`` (the mode set K(kmax), [M, 3] as (kx, ky, kz)), and the amplitudes
    of v and A, ``a_v``, ``c_v``, ``a_A``, ``c_A`` ([M, 3]: component d of the
    field is sum_k a[k, d] cos(2 pi k.x) + c[k, d] sin(2 pi k.x)), already scaled
    to the rms values; plus the density's ``kset_rho``, mode indices ``idx`` and
    phases ``phi``.  These amplitudes are the velocity and potential Fourier
    fields of the adjoint workload's control."""
    rng = np.random.Generator(np.random.PCG64(seed))
    kset_rho = mode_set(min(kmax, 4))
    kset = mode_set(kmax)
    idx = rng.integers(0, len(kset_rho), size=8)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=8)
    av = rng.standard_normal((len(kset), 3))
    cv = rng.standard_normal((len(kset), 3))
    aA = rng.standard_normal((len(kset), 3))
    cA = rng.standard_normal((len(kset), 3))
    # velocity: grid mean of |v|^2 is 1/2 sum_k (|a_k|^2 + |c_k|^2) (no aliasing for n > 2 kmax)
    msq = 0.5 * float(np.sum(av ** 2) + np.sum(cv ** 2))
    sv = v_rms / np.sqrt(msq) if v_rms > 0 else 0.0
    # potential: continuous curl of a cos(2 pi k.x) is -2 pi (k x a) sin(...), so
    # mean |curl A|^2 = 1/2 (2 pi)^2 sum_k (|k x a_k|^2 + |k x c_k|^2)
    kf = kset.astype(np.float64)
    cm = 0.5 * (2 * np.pi) ** 2 * float(np.sum(np.cross(kf, aA) ** 2) + np.sum(np.cross(kf, cA) ** 2))
    sA = b_rms / np.sqrt(cm) if b_rms > 0 else 0.0
    return dict(kset_rho=kset_rho, idx=idx, phi=phi, kset=kset, a_v=sv * av, c_v=sv * cv, a_A=sA * aA, c_A=sA * cA)


def evaluate_modes(n: int, ks: np.ndarray, a: np.ndarray, c: np.ndarray, offset) -> np.ndarray:
    """sum_k a_k cos(2 pi k.x) + c_k sin(2 pi k.x) on an n^3 grid at x = (idx +
    offset)/n (scalar amplitudes a, c of shape [M])."""
    return _evaluate(n, ks, a, c, offset)


def random_fields(n: int, seed: int, v_rms: float, kmax: int = 4, b_rms: float = 0.1,
                  B0=(1.0, 0.5, 0.0), P0: float = 0.6, gamma: float = 5.0 / 3.0, device=None) -> Fields:
    """Seeded random initial fields on an n^3 unit box (recipe in the module doc).
    With ``device`` (a torch device) the Fourier sums are evaluated there and the
    fields are float64 torch tensors on it (for large boxes)."""
    m = fourier_modes(seed, v_rms, kmax, b_rms)
    kset_rho, idx, phi, kset = m["kset_rho"], m["idx"], m["phi"], m["kset"]

    if device is not None:
        import torch
        ev = lambda *args: _evaluate_device(n, *args, device=device)
        stack = torch.stack
    else:
        ev = lambda *args: _evaluate(n, *args)
        stack = np.stack

    # density: 0.1 sin(theta + phi) = 0.1 (sin phi) cos theta + 0.1 (cos phi) sin theta
    ks_r = kset_rho[idx]
    rho = 1.0 + ev(ks_r, 0.1 * np.sin(phi), 0.1 * np.cos(phi), (0.5, 0.5, 0.5))

    v = stack([ev(kset, m["a_v"][:, d], m["c_v"][:, d], V_OFFSET) for d in range(3)])
    A = stack([ev(kset, m["a_A"][:, d], m["c_A"][:, d], EDGE_OFFSETS[d]) for d in range(3)])
    if device is not None:
        return Fields(rho=rho, v=v, A=A, B0=tuple(float(x) for x in B0), P0=float(P0), gamma=float(gamma))
    return Fields(rho=np.ascontiguousarray(rho), v=np.ascontiguousarray(v),
                  A=np.ascontiguousarray(A), B0=tuple(float(x) for x in B0), P0=float(P0),
                  gamma=float(gamma))


# Named workloads: grid, steps and generator parameters.
WORKLOADS = {
    # one FP64 step on 32^3, Mach 0.1, beta ~ 1
    "mach0.1_32": dict(n=32, steps=1, seed=1, v_rms=0.1, kmax=4, B0=(1.0, 0.5, 0.0)),
    # 10 FP64 steps on 256^3, Mach 2, beta ~ 1 (the throughput workload)
    "mach2_256": dict(n=256, steps=10, seed=1, v_rms=2.0, kmax=4, B0=(1.0, 0.5, 0.0)),
    # same generator sampled at 64^3: the oracle-sized version of the 256^3 run
    "mach2_64": dict(n=64, steps=10, seed=1, v_rms=2.0, kmax=4, B0=(1.0, 0.5, 0.0)),
    # mixed precision workload, Mach 0.1 inputs on 256^3
    "mixed_mach0.1_256": dict(n=256, steps=10, seed=1, v_rms=0.1, kmax=4, B0=(1.0, 0.5, 0.0)),
    # adjoint workload, Mach 1 on 128^3, 20 steps
    "adjoint_mach1_128": dict(n=128, steps=20, seed=1, v_rms=1.0, kmax=4, B0=(1.0, 0.5, 0.0)),
    # Mach 5 turbulence on 512^3, k <= 8, beta = 0.5
    "mach5_512": dict(n=512, steps=10, seed=1, v_rms=5.0, kmax=8,
                   B0=tuple(float(np.sqrt(2.4 / 1.25)) * x for x in (1.0, 0.5, 0.0))),
}


def workload_fields(name: str, n: int | None = None, seed: int | None = None) -> Fields:
    """Fields of a named workload, optionally resampled at another grid size/seed."""
    c = WORKLOADS[name]
    return random_fields(n or c["n"], seed if seed is not None else c["seed"], c["v_rms"],
                         kmax=c["kmax"], B0=c["B0"])


def fast_wave(nx: int, ny: int = 4, nz: int = 4, t: float = 0.0, A0: float = 1e-6, gamma: float = 5.0 / 3.0):
    """Grid-aligned linear fast wave of Sect. 4.1: Q = Qbar + A0 R_fast sin(2 pi (x - 2 t))
    on nx x ny x nz zones with h = 1/nx, using the right eigenvector the paper
    prints for Qbar = (1, 0,0,0, 1, sqrt2, 1/2, P = 1/gamma) (fast speed 2).
    Face b_y, b_z take the value at the zone-centre x; b_x = 1.  Returns the
    conserved state as numpy arrays: rho, m [3], E, b [3]."""
    s5 = 1.0 / (6.0 * np.sqrt(5.0))
    R = np.array([6, 12, -4 * np.sqrt(2.0), -2, 0, 8 * np.sqrt(2.0), 4, 27]) * s5
    x = (np.arange(nx) + 0.5) / nx
    s = np.broadcast_to(np.sin(2 * np.pi * (x - 2.0 * t)), (nz, ny, nx))
    Bb = (1.0, np.sqrt(2.0), 0.5)
    Eb = (1.0 / gamma) / (gamma - 1.0) + 0.5 * sum(q * q for q in Bb)
    return dict(rho=np.ascontiguousarray(1.0 + A0 * R[0] * s),
                m=np.ascontiguousarray(np.stack([A0 * R[1] * s, A0 * R[2] * s, A0 * R[3] * s])),
                E=np.ascontiguousarray(Eb + A0 * R[7] * s),
                b=np.ascontiguousarray(np.stack([np.ones_like(s), Bb[1] + A0 * R[5] * s, Bb[2] + A0 * R[6] * s])))


# ---------------------------------------------------------------------------
# oblique linear waves (Sect. 4.1, 3D setup)
# ---------------------------------------------------------------------------

_S5 = 1.0 / (6.0 * np.sqrt(5.0))
# right eigenvectors printed in Sect. 4.1 for the conserved variables (rho, m_1,
# m_2, m_3, B_1, B_2, B_3, E) in the wave frame, the wave speed, the background
# velocity along the wave vector and whether the background field is present
WAVE_MODES = {
    "fast": (np.array([6, 12, -4 * np.sqrt(2.0), -2, 0, 8 * np.sqrt(2.0), 4, 27]) * _S5, 2.0, 0.0, True),
    "slow": (np.array([12, 6, 8 * np.sqrt(2.0), 4, 0, -4 * np.sqrt(2.0), -2, 9]) * _S5, 0.5, 0.0, True),
    "alfven": (np.array([0, 0, 1, -2 * np.sqrt(2.0), 0, -1, 2 * np.sqrt(2.0), 0]) * _S5, 1.0, 0.0, True),
    "entropy": (np.array([1, 1, 0, 0, 0, 0, 0, 0.5]), 1.0, 1.0, True),
    "sound": (np.array([1, 1, 0, 0, 0, 0, 0, 1.5]), 1.0, 0.0, False),
    "shear": (np.array([0, 0, 1, 0, 0, 0, 0, 0]), 1.0, 1.0, False),
    "entropy_hydro": (np.array([1, 1, 0, 0, 0, 0, 0, 0.5]), 1.0, 1.0, False),
}


def wave_frame():
    """Unit vectors (e1, e2, e3) of the wave frame in lab coordinates: the
    columns of the rotation of Sect. 4.1 with sin(alpha) = 2/3 and the angle
    beta chosen so that the wave is periodic on the 3 x 1.5 x 1.5 box:
    e1 = (1/3, 2/3, 2/3) (one wavelength along every box edge)."""
    sa, ca = 2.0 / 3.0, np.sqrt(5.0) / 3.0
    sb, cb = 2.0 / np.sqrt(5.0), 1.0 / np.sqrt(5.0)
    e1 = np.array([ca * cb, ca * sb, sa])
    e2 = np.array([-sb, cb, 0.0])
    e3 = np.array([-sa * cb, -sa * sb, ca])
    return e1, e2, e3


def oblique_wave(N: int, mode: str, A0: float = 1e-6, t: float = 0.0, gamma: float = 5.0 / 3.0):
    """Linear wave of Sect. 4.1 propagating along e1 = (1/3, 2/3, 2/3) through a
    periodic 2N x N x N box of size 3 x 1.5 x 1.5 (zone size h = 1.5/N):
    Q = Qbar + A0 R_k sin(2 pi (x_1 - c t)) in the conserved variables, x_1 = e1 . r
    the zone-centre coordinate along the wave.  Background: rho = 1, P = 1/gamma,
    v = v_bg e1, B = e1 + sqrt(2) e2 + e3/2 for the MHD modes (B = 0 for the
    hydrodynamic ones).  The face field is b = B_bg + curl_h A with the edge
    potential A = -A0/(2 pi) R_B3 cos(2 pi x_1) e2 + A0/(2 pi) R_B2 cos(2 pi x_1) e3,
    whose curl is A0 (R_B2 e2 + R_B3 e3) sin(2 pi x_1), in phase with the other
    variables.  Returns the zone-centred conserved fields (rho, m [3], E), the
    potential on the edges (A [3], A_x at (i, j+1/2, k+1/2) ...), the uniform
    field B0, the zone size, the wave speed and the frame."""
    if mode not in WAVE_MODES:
        raise ValueError(f"unknown mode {mode}")
    R, c, vbg, mhd = WAVE_MODES[mode]
    if not mhd and mode == "sound":
        R = R.copy()
        R[7] = 1.0 / (gamma - 1.0)
    e1, e2, e3 = wave_frame()
    nx, ny, nz = 2 * N, N, N
    h = 1.5 / N

    def coord(offset):
        x = (np.arange(nx) + offset[0]) * h
        y = (np.arange(ny) + offset[1]) * h
        z = (np.arange(nz) + offset[2]) * h
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        return e1[0] * X + e1[1] * Y + e1[2] * Z

    x1 = coord((0.5, 0.5, 0.5))
    s = np.sin(2 * np.pi * (x1 - c * t))
    Bw = np.array([1.0, np.sqrt(2.0), 0.5]) if mhd else np.zeros(3)
    B0 = Bw[0] * e1 + Bw[1] * e2 + Bw[2] * e3
    rho = 1.0 + A0 * R[0] * s
    mw = [vbg + A0 * R[1] * s, A0 * R[2] * s, A0 * R[3] * s]
    m = np.stack([mw[0] * e1[d] + mw[1] * e2[d] + mw[2] * e3[d] for d in range(3)])
    Ebar = (1.0 / gamma) / (gamma - 1.0) + 0.5 * vbg * vbg + 0.5 * float(Bw @ Bw)
    E = Ebar + A0 * R[7] * s
    edge_offsets = [(0.5, 1.0, 1.0), (1.0, 0.5, 1.0), (1.0, 1.0, 0.5)]
    A = np.zeros((3, nz, ny, nx))
    if mhd:
        for d in range(3):
            cs = np.cos(2 * np.pi * (coord(edge_offsets[d]) - c * t))
            a2 = -A0 / (2 * np.pi) * R[6] * cs
            a3 = A0 / (2 * np.pi) * R[5] * cs
            A[d] = a2 * e2[d] + a3 * e3[d]
    return dict(rho=np.ascontiguousarray(rho), m=np.ascontiguousarray(m), E=np.ascontiguousarray(E),
                A=np.ascontiguousarray(A), B0=tuple(float(x) for x in B0), h=h, speed=c, shape=(nz, ny, nx),
                frame=(e1, e2, e3), gamma=gamma)

