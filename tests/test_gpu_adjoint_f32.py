"""The adjoint on an FP32-state patch (WM_MIXED_F32STATE): the state arguments
are float arrays, widened to FP64 on load, and the FP64 method is linearised at
the widened states; the stage states the adjoint recomputes come from the
FP32-state forward.

Bars:
  rhs VJP at a float state .............. <= 1e-10 of autograd through the
                                           oracle at the widened state
  step adjoint, stage states recomputed . <= 1e-13 of the FP64 patch's step
                                           adjoint given the same (widened)
                                           FP32-state stage states
  rollout gradient ...................... <= 1e-5 normwise of the FP64 rollout's
                                           (the two forwards differ by FP32
                                           rounding of the state, ~1e-7)
"""
import sys

import pytest
import torch

from oracle import mhd
from paper_1812_04278_amd import binding as B
from paper_1812_04278_amd import rollout as R
from helpers import fields, oracle_state, rel_err

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.load()


def flat8(U):
    return torch.stack([U["rho"], U["m"][0], U["m"][1], U["m"][2], U["E"], U["b"][0], U["b"][1], U["b"][2]])


def float_state(U):
    """The state rounded to FP32 (float tensors) and widened back (the oracle's dict)."""
    h = torch.stack([U["rho"], U["m"][0], U["m"][1], U["m"][2], U["E"]]).float().contiguous()
    b = U["b"].float().contiguous()
    hw, bw = h.double(), b.double()
    return h, b, dict(rho=hw[0], m=hw[1:4].clone(), E=hw[4], b=bw)


def check8(gpu, ref, label, tol):
    errs = [rel_err(gpu[c], ref[c]) for c in range(8)]
    say(f"  {label}: " + " ".join(f"{e:.1e}" for e in errs))
    assert max(errs) <= tol, (label, errs)


def test_f32_rhs_vjp_vs_oracle():
    say("FP32-state rhs vjp 37x21x19")
    f = fields(40, seed=12, v_rms=1.5, crop=(37, 21, 19))
    U, cfg = oracle_state(f)
    hf, bf, Uw = float_state(U)
    g = torch.Generator().manual_seed(3)
    lam = torch.randn((8,) + U["rho"].shape, generator=g, dtype=torch.float64)
    Ur = {k: v.clone().requires_grad_(True) for k, v in Uw.items()}
    s = (flat8(mhd.rhs(Ur, cfg)) * lam).sum()
    gr = torch.autograd.grad(s, [Ur["rho"], Ur["m"], Ur["E"], Ur["b"]])
    ref = torch.cat([gr[0][None], gr[1], gr[2][None], gr[3]])
    nz, ny, nx = U["rho"].shape
    p = B.Patch(B.config(nx=nx, ny=ny, nz=nz, h=cfg.h, precision=B.WM_MIXED_F32STATE))
    out = p.rhs_vjp(hf.cuda(), bf.cuda(), lam.cuda()).cpu()
    check8(out, ref, "FP32-state rhs vjp", 1e-10)


def test_f32_adjoint_step_recomputed_stages():
    """The step adjoint with recomputed stage states (FP32-state forward) equals
    the FP64 patch's adjoint given those stage states widened."""
    say("FP32-state adjoint step 20x18x16")
    f = fields(24, seed=13, v_rms=1.0, crop=(20, 18, 16))
    U, cfg = oracle_state(f)
    hf, bf, Uw = float_state(U)
    dt = 0.8 * mhd.compute_dt(Uw, cfg)
    nz, ny, nx = U["rho"].shape
    g = torch.Generator().manual_seed(4)
    lam = torch.randn((8, nz, ny, nx), generator=g, dtype=torch.float64).cuda()
    p32 = B.Patch(B.config(nx=nx, ny=ny, nz=nz, h=cfg.h, precision=B.WM_MIXED_F32STATE))
    p32.set_state(hf[0], hf[1:4], hf[4], bf)
    U1, U2 = p32.step_record(dt)                       # FP32 stage states of the mixed forward
    lh, lb = lam[:5].clone(), lam[5:].clone()
    p32.adjoint_step(hf.cuda(), bf.cuda(), dt, lh, lb)  # recomputes U1, U2 in FP32
    p64 = B.Patch(B.config(nx=nx, ny=ny, nz=nz, h=cfg.h))
    rh, rb = lam[:5].clone(), lam[5:].clone()
    p64.adjoint_step(hf.double().cuda(), bf.double().cuda(), dt, rh, rb, U1.double(), U2.double())
    check8(torch.cat([lh, lb]).cpu(), torch.cat([rh, rb]).cpu(), "recomputed vs given stages", 1e-13)
    # the recorded stage states passed in give the same result
    lh2, lb2 = lam[:5].clone(), lam[5:].clone()
    p32.adjoint_step(hf.cuda(), bf.cuda(), dt, lh2, lb2, U1, U2)
    check8(torch.cat([lh2, lb2]).cpu(), torch.cat([rh, rb]).cpu(), "given FP32 stages", 1e-13)


@pytest.mark.parametrize("integrator", [B.WM_SSPRK3, B.WM_RK4])
def test_f32_rollout_gradient_close_to_fp64(integrator):
    """Gradient of a final-state loss through the FP32-state rollout (mixed
    forward, FP64 adjoint at the widened states) against the FP64 rollout."""
    say(f"FP32-state rollout gradient, integrator {integrator}, 16^3, 6 steps")
    n = 16
    f = fields(n, seed=21, v_rms=1.0, kmax=2, B0=(1.0, 0.6, 0.8))
    cfl = 0.8 if integrator == B.WM_RK4 else 0.4
    grads = {}
    for prec in (B.WM_FP64, B.WM_MIXED_F32STATE):
        p = B.Patch(B.config(n, precision=prec, integrator=integrator, cfl=cfl))
        A = torch.as_tensor(f.A).cuda().requires_grad_(True)
        v = torch.as_tensor(f.v).cuda().requires_grad_(True)
        rho = torch.as_tensor(f.rho).cuda()
        hyd, bf, bc = R.rollout(A, v, rho, p, 6, ckpt_every=2, P0=f.P0, B0=f.B0)
        J = (hyd[0].double() ** 2).sum() + (0.5 * (bc.double() ** 2).sum(0) ** 2).sum()
        grads[prec] = torch.autograd.grad(J, [A, v])
    for i, name in enumerate(("A", "v")):
        a, b = grads[B.WM_MIXED_F32STATE][i], grads[B.WM_FP64][i]
        e = float((a - b).norm() / b.norm())
        say(f"  grad {name}: FP32-state vs FP64 {e:.2e}")
        assert torch.isfinite(a).all() and e <= 1e-5, (name, e)
