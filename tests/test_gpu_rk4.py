"""GPU parity of the classical RK4 integrator of Sect. 2.1 (the paper's own
time stepper, at its Courant number 0.8) against the oracle's q_save form.
The GPU takes the increment form U^n + dt/6 (k0 + 2 k1 + 2 k2 + k3), equal up
to rounding order.  Bar as for SSP-RK3: normwise relative difference per
variable <= 1e-12 in FP64."""
import dataclasses
import sys

import numpy as np
import pytest
import torch

from oracle import mhd
from paper_1812_04278_amd import binding as B
from helpers import assert_state_parity, fields, oracle_state, rel_err, state_errors

pytestmark = pytest.mark.gpu
TOL = 1e-12
CFL4 = 0.8


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.load()


def rk4_patch(f, h=None, **kw):
    nz, ny, nx = f.rho.shape
    p = B.Patch(B.config(nx=nx, ny=ny, nz=nz, h=h if h is not None else 1.0 / nx, cfl=CFL4,
                         integrator=B.WM_RK4, **kw))
    p.init_from_potential(f.rho, f.v, f.A, f.P0, f.B0)
    return p


def test_rk4_step_32():
    """One RK4 step on the 32^3 Mach-0.1 inputs, dt from each side's eq. (cfl) at CFL 0.8."""
    say("RK4 step 32^3")
    f = fields(32, seed=1, v_rms=0.1)
    U, cfg = oracle_state(f)
    cfg = dataclasses.replace(cfg, cfl=CFL4)
    p = rk4_patch(f)
    dt_g = p.step(want_dt=True)
    U1, dt_o = mhd.step_rk4(U, cfg)
    assert abs(dt_g - dt_o) <= 1e-14 * dt_o
    assert_state_parity(p.state(), U1, label="RK4 step")
    assert rel_err(p.bcell.cpu(), mhd.zone_B(U1["b"])) <= TOL


def test_rk4_three_steps_ragged_mach2():
    """Three Mach-2 RK4 steps on a ragged 37 x 21 x 19 crop of the 40^3 generator
    (h = 1/40), stages called one by one with the oracle's dt."""
    say("RK4 3 steps 37x21x19 Mach 2")
    f = fields(40, seed=4, v_rms=2.0, crop=(37, 21, 19))
    U, cfg = oracle_state(f, h=1.0 / 40)
    cfg = dataclasses.replace(cfg, cfl=CFL4)
    p = rk4_patch(f, h=1.0 / 40)
    for _ in range(3):
        U, dt = mhd.step_rk4(U, cfg)
        for s in range(4):
            p.rk_stage(s, dt)
    assert_state_parity(p.state(), U, label="RK4 ragged")


@pytest.mark.parametrize("n", [4, 5])
def test_rk4_tiny_grids(n):
    say(f"RK4 tiny grid {n}")
    f = fields(n, seed=7 + n, v_rms=0.5, kmax=1)
    U, cfg = oracle_state(f)
    cfg = dataclasses.replace(cfg, cfl=CFL4)
    p = rk4_patch(f)
    for _ in range(2):
        dt_g = p.step(want_dt=True)
        U, dt_o = mhd.step_rk4(U, cfg)
        assert abs(dt_g - dt_o) <= 1e-14 * dt_o
    assert_state_parity(p.state(), U, label=f"RK4 tiny {n}")


def test_rk4_mixed_one_step_32():
    """The mixed arithmetic under RK4: one step within the one-step bound of the
    SSP-RK3 mixed form (1e-8) of the FP64 oracle; FP32 state within 1e-6."""
    say("RK4 mixed / FP32 state, 32^3")
    f = fields(32, seed=1, v_rms=0.1)
    U, cfg = oracle_state(f)
    cfg = dataclasses.replace(cfg, cfl=CFL4)
    U1, dt = mhd.step_rk4(U, cfg)
    for prec, bound in ((B.WM_MIXED, 1e-8), (B.WM_MIXED_F32STATE, 1e-6)):
        p = rk4_patch(f, precision=prec)
        p.step_dt(dt)
        errs = state_errors(p.state(), U1)
        say("  ", prec, {k: f"{v:.2e}" for k, v in errs.items()})
        assert max(errs.values()) <= bound, (prec, errs)


def test_rk4_uniform_state_bitwise():
    n = 12
    ones = np.ones((n, n, n))
    v = np.stack([0.7 * ones, -0.4 * ones, 0.25 * ones])
    p = B.Patch(B.config(n, cfl=CFL4, integrator=B.WM_RK4))
    p.init_from_potential(1.3 * ones, v, np.zeros((3, n, n, n)), 0.6, (1.0, 0.5, -0.3))
    h0, b0 = p.hydro.clone(), p.bface.clone()
    for _ in range(2):
        p.step()
    torch.cuda.synchronize()
    assert torch.equal(p.hydro, h0) and torch.equal(p.bface, b0)


def test_rk4_stage_order_and_refusals():
    """Stage numbers outside the integrator's range are argument errors, stages out
    of order are state errors, stage recording refuses an RK4 patch and its step
    adjoint refuses stage states (it recomputes them)."""
    f = fields(8, seed=3, v_rms=0.3, kmax=2)
    p3 = B.Patch(B.config(8))
    p3.init_from_potential(f.rho, f.v, f.A, f.P0, f.B0)
    with pytest.raises(B.WmError) as e:
        p3.rk_stage(3, 1e-3)
    assert e.value.status == B.WM_ERR_ARG
    p = rk4_patch(f)
    with pytest.raises(B.WmError) as e:
        p.rk_stage(4, 1e-3)
    assert e.value.status == B.WM_ERR_ARG
    with pytest.raises(B.WmError) as e:
        p.rk_stage(1, 1e-3)
    assert e.value.status == B.WM_ERR_STATE
    with pytest.raises(B.WmError) as e:
        p.step_record(1e-3)
    assert e.value.status == B.WM_ERR_ARG
    lh = torch.zeros((5, 8, 8, 8), dtype=torch.float64, device="cuda")
    lb = torch.zeros((3, 8, 8, 8), dtype=torch.float64, device="cuda")
    S = torch.zeros((8, 8, 8, 8), dtype=torch.float64, device="cuda")
    with pytest.raises(B.WmError) as e:   # the RK4 step adjoint recomputes its stages
        p.adjoint_step(p.hydro.clone(), p.bface.clone(), 1e-3, lh, lb, S, S.clone())
    assert e.value.status == B.WM_ERR_ARG
    # a full step still runs after the refused calls
    p.step()
    assert p.diagnostics()["n_unphysical"] == 0
