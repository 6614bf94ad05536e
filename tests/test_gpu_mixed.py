"""Mixed precision (FP32 projections, split fluxes, weights, zone primitives and
transport-flux means; FP64 state, pressure recovery, eigen-system
renormalisation, differences and central flux) against the FP64 oracle and the
FP64 GPU path, and the order of convergence of both precisions on a smooth
grid-aligned fast wave (Sect. 4.1 setup, the paper's R_fast).

Stated bounds (normwise relative per variable, max|x - ref| / max|ref|):
  one step, 32^3 Mach 0.1 ........................ <= 1e-8  vs the oracle
  ten steps, 64^3 Mach 2 ......................... <= 1e-6  vs the oracle
  ten steps, 128^3 Mach 0.1 ...................... L1 per variable <= 1e-9 vs FP64
Measured (MI355X): 1.8e-9, 4.7e-8 and 1.1e-10 respectively.

FP32 state (WM_MIXED_F32STATE: the mixed arithmetic with hydro, face b, zone B,
stage states, accumulator and face fluxes stored in FP32; each store rounds to
~6e-8 relative):
  one step, 32^3 Mach 0.1 ........................ <= 1e-6  vs the oracle
  one step, 36 and 37 x 21 x 19 Mach 1 ........... <= 1e-6  vs the oracle (two-zone
                                                   and one-zone update)
  ten steps, 64^3 Mach 2 ......................... <= 2e-5  vs the oracle
  ten steps, 128^3 Mach 0.1 ...................... L1 per variable <= 1e-6 vs FP64
"""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import mhd
from paper_1812_04278_amd import binding as B
from helpers import _subbox, fields, oracle_state, state_errors
from paper_1812_04278_amd import inputs

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.load()


def patch(f, precision):
    nz, ny, nx = f.rho.shape
    p = B.Patch(B.config(nx=nx, ny=ny, nz=nz, h=1.0 / nx, precision=precision))
    p.init_from_potential(f.rho, f.v, f.A, f.P0, f.B0)
    return p


def test_mixed_one_step_32():
    say("mixed, one step 32^3 Mach 0.1")
    f = fields(32, seed=1, v_rms=0.1)
    U, cfg = oracle_state(f)
    p = patch(f, B.WM_MIXED)
    p.step()
    U1, _ = mhd.step(U, cfg)
    errs = state_errors(p.state(), U1)
    say("  ", {k: f"{v:.2e}" for k, v in errs.items()})
    assert max(errs.values()) <= 1e-8, errs


def test_mixed_wenoz_one_step_32():
    """Mixed precision with WENO-Z weights (evaluated in FP64: eps_Z = 1e-40 lies
    below the FP32 range), including a region of constant state where every
    smoothness indicator is zero."""
    import dataclasses
    say("mixed WENO-Z, one step 32^3 Mach 0.1 with a constant block")
    f = fields(32, seed=1, v_rms=0.1)
    f.v[:, 8:20, 8:20, :] = 0.0
    f.rho[8:20, 8:20, :] = 1.0
    f.A[:, 6:22, 6:22, :] = 0.0
    U, cfg = oracle_state(f)
    cfg = dataclasses.replace(cfg, weights="z")
    nz, ny, nx = f.rho.shape
    p = B.Patch(B.config(nx=nx, ny=ny, nz=nz, h=1.0 / nx, precision=B.WM_MIXED, weights=B.WM_WENO_Z))
    p.init_from_potential(f.rho, f.v, f.A, f.P0, f.B0)
    p.step()
    U1, _ = mhd.step(U, cfg)
    st = p.state()
    assert all(bool(torch.isfinite(torch.as_tensor(st[k])).all()) for k in st)
    errs = state_errors(st, U1)
    say("  ", {k: f"{v:.2e}" for k, v in errs.items()})
    assert max(errs.values()) <= 1e-8, errs


def test_mixed_ten_steps_64_mach2():
    say("mixed, 10 steps 64^3 Mach 2")
    f = fields(64, seed=1, v_rms=2.0)
    U, cfg = oracle_state(f)
    p = patch(f, B.WM_MIXED)
    for _ in range(10):
        p.step()
        U, _ = mhd.step(U, cfg)
    errs = state_errors(p.state(), U)
    say("  ", {k: f"{v:.2e}" for k, v in errs.items()})
    assert max(errs.values()) <= 1e-6, errs
    assert p.diagnostics()["max_divb"] <= 1e-12 * 64


def test_mixed_vs_fp64_l1_128():
    """L1 of the mixed run against the FP64 run (the Sect. 3 norm per variable)."""
    say("mixed vs fp64 L1, 128^3 Mach 0.1, 10 steps")
    f = fields(128, seed=1, v_rms=0.1)
    a, b = patch(f, B.WM_FP64), patch(f, B.WM_MIXED)
    for _ in range(10):
        dt = a.step(want_dt=True)
        b.step_dt(dt)
    per, geo = mhd.l1_error(a.state(), b.state())
    say("   L1 per variable", [f"{x:.2e}" for x in per], f"geometric {geo:.2e}")
    assert max(per) <= 1e-9


def fast_wave_k1(n, precision, A0, t_end=0.5, c=0.25):
    """Grid-aligned fast wave (Sect. 4.1 setup, the paper's R_fast) on n x 4 x 4
    zones, one period, dt = c h^(5/3).  Returns (L1 of Sect. 3 over the conserved
    variables, error of the k = 1 Fourier amplitudes) against the exact
    travelling wave."""
    U0, U1 = inputs.fast_wave(n, A0=A0), inputs.fast_wave(n, t=t_end, A0=A0)
    p = B.Patch(B.config(nx=n, ny=4, nz=4, h=1.0 / n, precision=precision))
    p.set_state(U0["rho"], U0["m"], U0["E"], U0["b"])
    nt = int(math.ceil(t_end / (c * (1.0 / n) ** (5.0 / 3.0))))
    for _ in range(nt):
        p.step_dt(t_end / nt)
    st = p.state()
    comps = lambda U: [np.asarray(x) for x in (U["rho"], U["m"][0], U["m"][1], U["m"][2], U["E"],
                                                U["b"][0], U["b"][1], U["b"][2])]
    l1 = math.sqrt(sum(float(np.abs(x - y).mean()) ** 2 for x, y in zip(comps(st), comps(U1))))
    k1 = lambda U: np.array([np.fft.rfft(x.mean(axis=(0, 1)))[1] / n for x in comps(U)])
    return l1, float(np.linalg.norm(k1(st) - k1(U1)))


def test_fast_wave_order_both_precisions():
    """Fifth order in both precisions.  The k = 1 Fourier amplitudes (A0 = 1e-5),
    which nonlinearity changes only at O(A0^3), converge at order ~5 from N = 32
    to 128; the L1 against the linear solution (A0 = 1e-6) reaches the O(A0^2)
    steepening floor (~3e-12) near N = 64, the limit Sect. 4.1 also reports for
    1D waves, so its order is asserted from 16 to 32.  The mixed errors equal the
    FP64 errors at these N."""
    res = {}
    for precision, name in ((B.WM_FP64, "fp64"), (B.WM_MIXED, "mixed")):
        k1 = [fast_wave_k1(n, precision, 1e-5)[1] for n in (32, 64, 128)]
        l1 = [fast_wave_k1(n, precision, 1e-6)[0] for n in (16, 32)]
        ko = [math.log2(k1[i] / k1[i + 1]) for i in range(2)]
        lo = math.log2(l1[0] / l1[1])
        say(f"fast wave {name}: k1 {[f'{e:.3e}' for e in k1]} orders {[f'{o:.2f}' for o in ko]}; "
            f"L1 {[f'{e:.3e}' for e in l1]} order {lo:.2f}")
        assert min(ko) > 4.8 and lo > 4.8, (name, k1, l1)
        res[name] = k1 + l1
    for a, b in zip(res["fp64"], res["mixed"]):
        assert abs(a - b) <= 2e-2 * a


def test_f32state_one_step_32():
    say("FP32 state, one step 32^3 Mach 0.1")
    f = fields(32, seed=1, v_rms=0.1)
    U, cfg = oracle_state(f)
    p = patch(f, B.WM_MIXED_F32STATE)
    assert p.hydro.dtype == torch.float32
    dt = p.step(want_dt=True)
    U1, dt_o = mhd.step(U, cfg)
    assert abs(dt - dt_o) <= 1e-6 * dt_o
    errs = state_errors(p.state(), U1)
    say("  ", {k: f"{v:.2e}" for k, v in errs.items()})
    assert max(errs.values()) <= 1e-6, errs


@pytest.mark.parametrize("nx", [36, 37])
def test_f32state_one_step_ragged(nx):
    """FP32 state on a ragged box (nx x 21 x 19, Mach ~1): with nx even the
    update takes two x-adjacent zones per thread (8-byte loads), with nx odd one;
    both against the oracle stepped from the same FP32-rounded state."""
    say(f"FP32 state, one step {nx}x21x19")
    f = fields(40, seed=7, v_rms=1.0, crop=(nx, 21, 19))
    U, cfg = oracle_state(f)
    Uf = {k: v.float().double() for k, v in U.items()}
    p = B.Patch(B.config(nx=nx, ny=21, nz=19, h=cfg.h, precision=B.WM_MIXED_F32STATE))
    p.set_state(Uf["rho"], Uf["m"], Uf["E"], Uf["b"])
    dt = 0.8 * mhd.compute_dt(Uf, cfg)
    p.step_dt(dt)
    U1, _ = mhd.step(Uf, cfg, dt)
    errs = state_errors(p.state(), U1)
    say("  ", {k: f"{v:.2e}" for k, v in errs.items()})
    assert max(errs.values()) <= 1e-6, errs


def test_f32state_ten_steps_64_mach2():
    say("FP32 state, 10 steps 64^3 Mach 2")
    f = fields(64, seed=1, v_rms=2.0)
    U, cfg = oracle_state(f)
    p = patch(f, B.WM_MIXED_F32STATE)
    for _ in range(10):
        U, dt = mhd.step(U, cfg)
        p.step_dt(dt)
    errs = state_errors(p.state(), U)
    say("  ", {k: f"{v:.2e}" for k, v in errs.items()})
    assert max(errs.values()) <= 2e-5, errs
    d = p.diagnostics()
    say(f"   max div b {d['max_divb']:.2e}")
    assert d["max_divb"] <= 1e-4


def test_f32state_vs_fp64_l1_128():
    say("FP32 state vs FP64 L1, 128^3 Mach 0.1, 10 steps")
    f = fields(128, seed=1, v_rms=0.1)
    a, b = patch(f, B.WM_FP64), patch(f, B.WM_MIXED_F32STATE)
    for _ in range(10):
        dt = a.step(want_dt=True)
        b.step_dt(dt)
    per, geo = mhd.l1_error(a.state(), b.state())
    say("   L1 per variable", [f"{x:.2e}" for x in per], f"geometric {geo:.2e}")
    assert max(per) <= 1e-6


def test_f32state_stage_record_and_adjoint_types():
    """Stage recording keeps the FP32 state type; the adjoint calls of an
    FP32-state patch take float state arrays (widened inside the library) and a
    zero cotangent gives a zero gradient."""
    f = fields(16, seed=2, v_rms=0.5)
    p = patch(f, B.WM_MIXED_F32STATE)
    U1, U2 = p.step_record(1e-3)
    assert U1.dtype == torch.float32 and bool(torch.isfinite(U1).all()) and bool(torch.isfinite(U2).all())
    lam = torch.zeros((8, 16, 16, 16), dtype=torch.float64, device="cuda")
    out = p.rhs_vjp(p.hydro, p.bface, lam)
    assert out.dtype == torch.float64 and float(out.abs().max()) == 0.0


def test_f32state_sampled_512_mach5():
    """The 512^3 Mach-5 workload (|k| <= 8, beta 0.5) in the FP32-state form, as
    the benchmark's 512^3 leg runs it: dt of eq. (cfl) against the oracle on the
    full box, and one GPU step checked at sampled zones against the FP64 oracle
    stepped on a periodic 48^3 sub-box of the same (FP32) state around each
    sample (dependence radius 18 < 24).  Bar: the FP32-state one-step bound,
    1e-6 of the sub-box's largest value per variable.  At this size the face
    arrays span 21 x 2^27 values, past 32-bit indexing."""
    import math
    n = 512
    B0 = tuple(math.sqrt(2.4 / 1.25) * x for x in (1.0, 0.5, 0.0))
    say("FP32 state 512^3 Mach 5: generating inputs")
    f = fields(n, seed=1, v_rms=5.0, kmax=8, B0=B0)
    p = patch(f, B.WM_MIXED_F32STATE)
    del f
    st0 = p.state()                       # float64 copy of the FP32 state
    dt = p.compute_dt()
    dt_o = mhd.compute_dt(st0, mhd.cubic(n))
    say(f"  dt gpu {dt:.9e} oracle {dt_o:.9e}")
    # the GPU reads the zone field it stores in FP32; the oracle interpolates it
    # from the faces in FP64 (FP32 rounding of B, ~6e-8, enters c_fast)
    assert abs(dt - dt_o) <= 1e-6 * dt_o
    p.step_dt(dt_o)
    st1 = p.state()
    assert p.diagnostics()["n_unphysical"] == 0
    g = torch.Generator().manual_seed(21)
    cents = [tuple(int(x) for x in torch.randint(0, n, (3,), generator=g)) for _ in range(3)]
    cfg48 = mhd.Config(48, 48, 48, 1.0 / n)
    for c in cents:
        sub = {key: _subbox(st0[key], c, 24) for key in st0}
        U1, _ = mhd.step(sub, cfg48, dt_o)
        for key in ("rho", "m", "E", "b"):
            gv = _subbox(st1[key], c, 24)[..., 20:28, 20:28, 20:28]
            ov = U1[key][..., 20:28, 20:28, 20:28]
            err = float((gv - ov).abs().max()) / float(ov.abs().max())
            assert err <= 1e-6, (c, key, err)
        say(f"  sample {c} ok")
