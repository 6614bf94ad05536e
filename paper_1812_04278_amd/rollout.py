"""Differentiable rollout: n steps of the patch's integrator (SSP-RK3 or the
classical RK4) from an initial vector potential and velocity, as a
``torch.autograd.Function`` whose backward runs the hand-written adjoint of the
HIP library (``wm_adjoint_step``, ``wm_init_adjoint``).

A patch with an FP32 state (WM_MIXED_F32STATE) runs the mixed forward and keeps
FP32 checkpoints; its backward linearises the FP64 method at those states
widened to FP64 (the cotangents are FP64 throughout).

Memory: the forward keeps a checkpoint of the state every ``ckpt_every`` steps;
the backward re-runs each segment forward from its checkpoint, keeping that
segment's states (and, with ``store_stages``, the two intermediate RK stages of
every step but the segment's last, so the adjoint step does not recompute them:
3 states of 8 fields per step of the segment; SSP-RK3 only -- the RK4 adjoint
recomputes its three stage states), and walks it in reverse.  The segment's last
step is not run forward: its adjoint step recomputes its two stage states, which
saves the third stage, whose result is the next checkpoint.  The forward pass keeps the states of
the last segment as it computes them (``keep_last``), so the backward starts
without re-running that segment.  The time steps of the forward pass are
recorded and held fixed in the backward (dt is not differentiated).
"""
from __future__ import annotations

import torch

from . import binding as B


class Rollout(torch.autograd.Function):
    """outputs = (hydro_T [5, ...], bface_T [3, ...], bcell_T [3, ...]) after
    ``nsteps`` steps from init_from_potential(rho, v, A, P0, B0)."""

    @staticmethod
    def forward(ctx, A, v, rho, patch: B.Patch, nsteps: int, ckpt_every: int, P0: float, B0, store_stages=True,
                keep_last=True):
        caller = torch.cuda.current_stream(patch.device)
        patch.stream.wait_stream(caller)        # the inputs are ready on the caller's stream
        store_stages = store_stages and patch.cfg.integrator == B.WM_SSPRK3
        last0 = (nsteps - 1) // ckpt_every * ckpt_every if keep_last and nsteps > 0 else nsteps
        with torch.no_grad(), torch.cuda.stream(patch.stream):
            patch.init_from_potential(rho, v, A, P0, B0)
            ckpts, dts, last = [], [], []
            for n in range(nsteps):
                if n % ckpt_every == 0:
                    ckpts.append((patch.hydro.clone(), patch.bface.clone()))
                if n < last0:
                    dts.append(patch.step(want_dt=True))
                    continue
                # the last segment: keep what its adjoint steps need
                Uh, Ub = patch.hydro.clone(), patch.bface.clone()
                if store_stages:
                    dts.append(patch.compute_dt())
                    U1, U2 = patch.step_record(dts[-1])
                else:
                    dts.append(patch.step(want_dt=True))
                    U1 = U2 = None
                last.append((Uh, Ub, U1, U2))
            out = (patch.hydro.clone(), patch.bface.clone(), patch.bcell.clone())
        for t in out:                           # made on the patch's stream, used on the caller's
            t.record_stream(caller)
        ctx.patch, ctx.nsteps, ctx.ckpt_every = patch, nsteps, ckpt_every
        ctx.ckpts, ctx.dts, ctx.P0, ctx.B0 = ckpts, dts, P0, B0
        ctx.store_stages = store_stages
        ctx.last = last
        ctx.save_for_backward(A, v, rho)
        caller.wait_stream(patch.stream)        # the outputs are ready on the patch's stream
        return out

    @staticmethod
    def backward(ctx, g_hydro, g_bface, g_bcell):
        A, v, rho = ctx.saved_tensors
        p = ctx.patch
        shape = p.shape
        dev = p.device
        caller = torch.cuda.current_stream(dev)
        p.stream.wait_stream(caller)
        with torch.no_grad(), torch.cuda.stream(p.stream):
            lam_h = (g_hydro if g_hydro is not None else torch.zeros((5,) + shape, dtype=torch.float64, device=dev))
            lam_b = (g_bface if g_bface is not None else torch.zeros((3,) + shape, dtype=torch.float64, device=dev))
            lam_h = lam_h.to(dev, torch.float64).contiguous().clone()
            lam_b = lam_b.to(dev, torch.float64).contiguous().clone()
            if g_bcell is not None:
                p.zone_field_vjp(g_bcell.to(dev, torch.float64), lam_b)
            n_seg = len(ctx.ckpts)
            for sgi in range(n_seg - 1, -1, -1):
                n0 = sgi * ctx.ckpt_every
                n1 = min(n0 + ctx.ckpt_every, ctx.nsteps)
                if sgi == n_seg - 1 and ctx.last:
                    states, ctx.last = ctx.last, []     # kept by the forward pass
                    n_run = 0
                else:
                    h0, b0 = ctx.ckpts[sgi]
                    # recompute the segment's states from its checkpoint with the recorded dts
                    p.set_state(h0[0], h0[1:4], h0[4], b0)
                    states = []
                    n_run = n1 - n0
                for n in range(n0, n0 + n_run):
                    Uh, Ub = p.hydro.clone(), p.bface.clone()
                    if ctx.store_stages and n + 1 < n1:
                        U1, U2 = p.step_record(ctx.dts[n])
                    else:
                        # the segment's last step (or every step without stored
                        # stages): the adjoint step recomputes its stage states,
                        # and the step's result, the next checkpoint, is not needed
                        U1 = U2 = None
                        if n + 1 < n1:
                            p.step_dt(ctx.dts[n])
                    states.append((Uh, Ub, U1, U2))
                for n in range(n1 - 1, n0 - 1, -1):
                    Uh, Ub, U1, U2 = states[n - n0]
                    p.adjoint_step(Uh, Ub, ctx.dts[n], lam_h, lam_b, U1, U2)
                del states
            gA, gv = p.init_adjoint(rho, v, A, ctx.B0, lam_h, lam_b)
        for t in (gA, gv):
            t.record_stream(caller)
        caller.wait_stream(p.stream)
        return gA, gv, None, None, None, None, None, None, None, None


def rollout(A, v, rho, patch: B.Patch, nsteps: int, ckpt_every: int = 5, P0: float = 0.6, B0=(1.0, 0.5, 0.0),
            store_stages: bool = True, keep_last: bool = True):
    return Rollout.apply(A, v, rho, patch, nsteps, ckpt_every, P0, B0, store_stages, keep_last)
