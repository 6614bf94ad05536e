#!/usr/bin/env python3
"""Throughput of the WENO5-CT MHD step on one MI355X.

Workload (default): 256^3 periodic box, seeded Mach-2 inputs (beta ~ 1),
SSP-RK3 steps at CFL 0.4 in FP64.  A step is the whole hot path: the time
step reduction and three stages (three directional sweeps, the divergence /
corner-flux / RK update and the zone-field interpolation each).  The state is
resident in HBM before the timed region; no host transfer inside it.

Prints one JSON line.  `value` is Mzone-updates/s = N^3 * steps / wall.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Mzone-updates/s per RK3 step, FP64 vs mixed at stated L1 err; adjoint/fwd cost"

# Algorithmic work of one sweep per face (FP64 flops): the count for the
# characteristic WENO5 flux of a face, ~2,100 (eigen-system 240, ten 7x7
# projections 980, split 140, 14 phi_N 560, central term and back-projection
# 130, transport flux 8), plus ~70 for the zone prologue (primitives, flux,
# eigenvalues) of the face's zone.
FLOPS_PER_FACE = 2170
# Algorithmic HBM traffic of the update kernel per zone, in stored values
# averaged over the three SSP-RK3 stages: reads 15 face fluxes, 6 transport
# fluxes, U^n (8) and the accumulator (8, stages 1-2); writes the stage state
# (8) and the accumulator (8, stages 0-1).  Times 8 bytes (FP64) or 4 (FP32 state).
UPDATE_VALUES_PER_ZONE = 21 + 8 + 8 * 2 / 3 + 8 + 8 * 2 / 3
PEAK_FP64_TFLOPS = 78.6
PEAK_HBM_GBS = 8000.0
# HBM bytes per sweep dispatch on the 256^3 FP64 workload, averaged over the
# three axes: FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 (the factors a plain copy of
# known size gives), profiles/fp64_step_256cube_pmc_traffic.md.
SWEEP_TRAFFIC_BYTES_256 = 2.221e9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def host_cpu():
    """CPU model and logical CPU count of the host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return model, os.cpu_count()


def cpu_baseline(threads: int | None = None):
    """The oracle as it stands, timed on the host cores on samples of the
    workloads: 32^3 Mach 0.1 with one SSP-RK3 step, and the Mach-2 generator
    sampled at 64^3 with ten steps, with all the threads torch uses; then the
    32^3 step and one 64^3 Mach-2 step on a single thread.  `value` is the 64^3
    Mach-2 rate (the Mach-2 workload's per-zone work)."""
    import torch
    from oracle import mhd
    from paper_1812_04278_amd import inputs

    def run(n, steps, v_rms):
        f = inputs.random_fields(n, seed=1, v_rms=v_rms, kmax=4)
        cfg = mhd.cubic(n)
        U = mhd.init_from_potential(f.rho, f.v, f.A, f.P0, f.B0, cfg)
        t0 = time.perf_counter()
        for _ in range(steps):
            U, _ = mhd.step(U, cfg)
        el = time.perf_counter() - t0
        return {"sample": f"{n}^3 x {steps} step(s), Mach {v_rms:g}", "seconds": round(el, 3),
                "value": round(n ** 3 * steps / el / 1e6, 6)}

    model, nproc = host_cpu()
    saved = torch.get_num_threads()
    if threads:
        torch.set_num_threads(threads)
    nthr = torch.get_num_threads()
    s32 = run(32, 1, 0.1)
    s64 = run(64, 10, 2.0)
    torch.set_num_threads(1)
    try:
        s32_1 = run(32, 1, 0.1)
        s64_1 = run(64, 1, 2.0)
    finally:
        torch.set_num_threads(saved)
    return dict(value=s64["value"], unit="Mzone-updates/s", cores=nthr, kind="oracle",
                sample=f"the Mach-2 generator sampled at 64^3 (seed 1), 10 SSP-RK3 steps, "
                       f"{s64['seconds']:.1f} s on {nthr} threads",
                host={"cpu_model": model, "nproc": nproc, "threads_used": nthr},
                samples={"mach0.1_32x1": s32, "mach2_64x10": s64},
                single_thread={"mach0.1_32x1": s32_1, "mach2_64x1": s64_1})


def l1_per_variable(a: dict, b: dict):
    """L1 of Sect. 3 per conserved variable (rho, m_x, m_y, m_z, E, b_x, b_y, b_z)
    and its geometric norm, between two GPU states (dicts of host tensors)."""
    comps = lambda U: [U["rho"], U["m"][0], U["m"][1], U["m"][2], U["E"], U["b"][0], U["b"][1], U["b"][2]]
    per = [float((x - y).abs().mean()) for x, y in zip(comps(a), comps(b))]
    return per, sum(v * v for v in per) ** 0.5


def timed_steps(p, steps: int, dts=None):
    """Runs `steps` steps (dt from eq. (cfl), or the given list) and returns (ms, dts)."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        if dts is None:
            p.step()
        else:
            p.step_dt(dts[s])
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3


def mixed_precision(n: int, steps: int):
    """The Mach-0.1 workload in FP64, in mixed precision (FP64 state) and in the
    mixed form with an FP32 state: throughput of each (own dt from eq. (cfl),
    HIP-event kernel times), and the L1 of the two mixed states against the
    FP64 state after `steps` steps taken with the FP64 run's dt sequence."""
    import torch
    from paper_1812_04278_amd import binding, inputs
    f = inputs.random_fields(n, seed=1, v_rms=0.1, kmax=4)
    res, states, dts = {}, {}, []
    for name, prec in (("fp64", binding.WM_FP64), ("mixed", binding.WM_MIXED),
                       ("f32state", binding.WM_MIXED_F32STATE)):
        p = binding.Patch(binding.config(n, precision=prec), device="cuda:0")
        p.init_from_potential(f.rho, f.v, f.A, f.P0, f.B0)
        p.step()                                    # warm-up
        p.init_from_potential(f.rho, f.v, f.A, f.P0, f.B0)
        p.profile(True)
        ms = timed_steps(p, steps)
        rep = p.profile_report()
        p.profile(False)
        nsw, msw = rep["sweep"]
        nup, msup = rep["update"]
        sw_ms, up_ms = msw / max(nsw, 1), msup / max(nup, 1)
        es = 4 if prec == binding.WM_MIXED_F32STATE else 8
        upd_bytes = UPDATE_VALUES_PER_ZONE * es * float(n) ** 3
        tf = FLOPS_PER_FACE * float(n) ** 3 / (sw_ms * 1e-3) / 1e12
        # sweep fraction against the FP64 vector peak in all three forms: with packed
        # FP32 instructions off, an FP32 vector instruction issues at the FP64 rate
        res[name] = {"value": round(n ** 3 * steps / (ms * 1e-3) / 1e6, 3), "ms_per_step": round(ms / steps, 4),
                     "sweep_avg_ms": round(sw_ms, 4), "sweep_tflops": round(tf, 3),
                     "sweep_frac_fp64_vector_peak": round(tf / PEAK_FP64_TFLOPS, 4),
                     "update_avg_ms": round(up_ms, 4),
                     "update_hbm_gbs": round(upd_bytes / (up_ms * 1e-3) / 1e9, 1),
                     "update_hbm_frac": round(upd_bytes / (up_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4)}
        # accuracy run: the FP64 dt sequence for both
        p.init_from_potential(f.rho, f.v, f.A, f.P0, f.B0)
        for s in range(steps):
            if name == "fp64":
                dts.append(p.step(want_dt=True))
            else:
                p.step_dt(dts[s])
        states[name] = p.state()
        del p
    per, geo = l1_per_variable(states["fp64"], states["mixed"])
    res["speedup"] = round(res["mixed"]["value"] / res["fp64"]["value"], 4)
    res["l1_mixed_vs_fp64"] = {"per_variable": [float(f"{x:.3e}") for x in per],
                               "variables": ["rho", "m_x", "m_y", "m_z", "E", "b_x", "b_y", "b_z"],
                               "geometric": float(f"{geo:.3e}")}
    # the mixed arithmetic with the state, stage states, accumulator and face
    # fluxes stored in FP32 (the form of the 512^3 workload)
    per, geo = l1_per_variable(states["fp64"], states["f32state"])
    res["speedup_f32state"] = round(res["f32state"]["value"] / res["fp64"]["value"], 4)
    res["l1_f32state_vs_fp64"] = {"per_variable": [float(f"{x:.3e}") for x in per], "geometric": float(f"{geo:.3e}")}
    res["workload"] = f"{n}^3 periodic box, Mach 0.1, beta~1, {steps} SSP-RK3 steps"
    return res


def convergence(sizes, c: float = 0.25):
    """Grid-aligned linear fast wave (Sect. 4.1 setup), one period, dt = c h^(5/3),
    on n x 4 x 4 zones, FP64 and mixed (SSP-RK3), and FP64 with the classical
    RK4 at the paper's Courant number 0.8.  Two errors against the exact
    travelling wave: the L1 of Sect. 3 (A0 = 1e-6; it meets the O(A0^2)
    nonlinear floor near N = 64) and the error of the k = 1 Fourier amplitude of
    every conserved variable (A0 = 1e-5), which nonlinearity changes only at
    O(A0^3) and so shows the truncation order further."""
    import math
    import numpy as np
    import torch
    from paper_1812_04278_amd import binding, inputs

    def k1(U):
        comps = [U["rho"], U["m"][0], U["m"][1], U["m"][2], U["E"], U["b"][0], U["b"][1], U["b"][2]]
        return np.array([np.fft.rfft(np.asarray(x, dtype=np.float64).mean(axis=(0, 1)))[1] / x.shape[-1]
                         for x in comps])

    out = {}
    runs = (("fp64", binding.WM_FP64, binding.WM_SSPRK3), ("mixed", binding.WM_MIXED, binding.WM_SSPRK3),
            ("fp64_rk4", binding.WM_FP64, binding.WM_RK4))
    for name, prec, integ in runs:
        l1, fk = [], []
        for n in sizes:
            for A0 in (1e-6, 1e-5):
                U0, U1 = inputs.fast_wave(n, A0=A0), inputs.fast_wave(n, t=0.5, A0=A0)
                p = binding.Patch(binding.config(nx=n, ny=4, nz=4, h=1.0 / n, precision=prec, integrator=integ),
                                  device="cuda:0")
                p.set_state(U0["rho"], U0["m"], U0["E"], U0["b"])
                if integ == binding.WM_RK4:   # the paper's setting: Courant number c_f dt / h = 0.8, c_f = 2
                    nt = int(math.ceil(0.5 / (0.4 / n)))
                else:
                    nt = int(math.ceil(0.5 / (c * (1.0 / n) ** (5.0 / 3.0))))
                for _ in range(nt):
                    p.step_dt(0.5 / nt)
                st = p.state()
                if A0 == 1e-6:
                    ex = {k: torch.as_tensor(v) for k, v in U1.items()}
                    l1.append(float(f"{l1_per_variable(st, ex)[1]:.4e}"))
                else:
                    fk.append(float(f"{np.linalg.norm(k1(st) - k1(U1)):.4e}"))
                del p
        out[name] = {"l1": l1, "l1_order": [round(math.log2(l1[i] / l1[i + 1]), 3) for i in range(len(l1) - 1)],
                     "k1": fk, "k1_order": [round(math.log2(fk[i] / fk[i + 1]), 3) for i in range(len(fk) - 1)]}
    out["sizes"] = list(sizes)
    return out


def rk4_leg(n: int, steps: int):
    """The headline workload (n^3, Mach 2, FP64) with the paper's classical RK4
    at CFL 0.8 next to SSP-RK3 at CFL 0.4, and the paper's own scheme (RK4 at
    CFL 0.8 with the WENO-Z weights): zone-updates per second per step of each,
    and simulated time advanced per wall-clock second (dt from eq. (cfl) each
    step, read back after the step)."""
    import torch
    from paper_1812_04278_amd import binding, inputs
    f = inputs.random_fields(n, seed=1, v_rms=2.0, kmax=4)
    out = {}
    for name, integ, cfl, w in (("rk4", binding.WM_RK4, 0.8, binding.WM_WENO_JS),
                                ("ssprk3", binding.WM_SSPRK3, 0.4, binding.WM_WENO_JS),
                                ("rk4_wenoz", binding.WM_RK4, 0.8, binding.WM_WENO_Z)):
        p = binding.Patch(binding.config(n, cfl=cfl, integrator=integ, weights=w), device="cuda:0")
        p.init_from_potential(f.rho, f.v, f.A, f.P0, f.B0)
        p.step()                                    # warm-up
        p.init_from_potential(f.rho, f.v, f.A, f.P0, f.B0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t_sim = 0.0
        for _ in range(steps):
            t_sim += p.step(want_dt=True)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        out[name] = {"value": round(n ** 3 * steps / wall / 1e6, 3), "unit": "Mzone-updates/s",
                     "ms_per_step": round(wall * 1e3 / steps, 4), "cfl": cfl, "sim_time": float(f"{t_sim:.6e}"),
                     "sim_time_per_wall_s": float(f"{t_sim / wall:.6e}")}
        del p
    out["sim_time_rate_rk4_vs_ssprk3"] = round(out["rk4"]["sim_time_per_wall_s"] / out["ssprk3"]["sim_time_per_wall_s"], 4)
    out["workload"] = (f"{n}^3 periodic box, Mach 2, beta~1, FP64, {steps} steps of each integrator "
                       "(Jiang-Shu weights; rk4_wenoz: the paper's RK4 with WENO-Z weights)")
    return out


def oblique_waves(sizes, modes=("fast", "slow", "alfven", "entropy"), t_end: float = 2.0, weights: str = "z"):
    """The 3D linear-wave suite of Sect. 4.1 with the paper's WENO-Z weights
    (weights: 'z' the reading R13, 'z_printed' as Sect. 2.2 prints them, 'js'
    Jiang-Shu) and RK4 at CFL 0.8: each MHD mode travels along (1, 2, 2)/3 through a 2N x N x N
    box (3 x 1.5 x 1.5).  Reports the L1 of Sect. 3 (rho, m, zone B, E; geometric
    norm) against the initial state after one wave period, and the decay rate of
    eq. (decay_rate) of the transverse field B_2 (wave frame) between t = 0 and
    t_end, with the convergence orders between successive N.  dt: the largest
    step within CFL 0.8 at t = 0 that divides the period."""
    import math
    import numpy as np
    import torch
    from paper_1812_04278_amd import binding, inputs

    def zone_vars(p):
        h = p.hydro.double()
        B = p.bcell.double()
        return [h[0], h[1], h[2], h[3], B[0], B[1], B[2], h[4]]

    def rms_B2(p, e2, bg):
        B = p.bcell.double()
        comp = B[0] * float(e2[0]) + B[1] * float(e2[1]) + B[2] * float(e2[2])
        return float(((comp - bg) ** 2).mean().sqrt())

    wcode = {"z": binding.WM_WENO_Z, "z_printed": binding.WM_WENO_Z_PRINTED, "js": binding.WM_WENO_JS}[weights]
    out = {"sizes": list(sizes), "t_end": t_end, "weights": weights, "integrator": "rk4", "cfl": 0.8}
    for mode in modes:
        l1, tau = [], []
        for N in sizes:
            w = inputs.oblique_wave(N, mode)
            nz, ny, nx = w["shape"]
            p = binding.Patch(binding.config(nx=nx, ny=ny, nz=nz, h=w["h"], cfl=0.8, weights=wcode,
                                             integrator=binding.WM_RK4), device="cuda:0")
            p.init_from_potential(w["rho"], np.zeros((3, nz, ny, nx)), w["A"], 1.0 / w["gamma"], w["B0"])
            p.set_state(w["rho"], w["m"], w["E"], p.bface)
            e2 = w["frame"][1]
            bg = math.sqrt(2.0)
            period = 1.0 / w["speed"]
            nt = int(math.ceil(period / p.compute_dt()))
            dt = period / nt
            ref = [x.clone() for x in zone_vars(p)]
            r0 = rms_B2(p, e2, bg)
            n_end = int(round(t_end / dt))
            for s in range(1, n_end + 1):
                p.step_dt(dt)
                if s == nt:
                    per = [float((x - y).abs().mean()) for x, y in zip(zone_vars(p), ref)]
                    l1.append(float(f"{math.sqrt(sum(v * v for v in per)):.4e}"))
            tau.append(float(f"{-math.log(rms_B2(p, e2, bg) / r0) / (n_end * dt):.4e}") if r0 > 0 else None)
            del p
        entry = {"l1": l1, "l1_order": [round(math.log2(l1[i] / l1[i + 1]), 3) for i in range(len(l1) - 1)]}
        if all(t is not None and t > 0 for t in tau):
            entry["decay_rate"] = tau
            entry["decay_rate_order"] = [round(math.log2(tau[i] / tau[i + 1]), 3) for i in range(len(tau) - 1)]
        out[mode] = entry
    return out


def adjoint_cost(n: int = 128, steps: int = 20, ckpt: int = 5):
    """The adjoint workload: gradient of J = h^3 sum[(rho_T - rho*)^2 + (|B_T|^2/2
    - e*)^2] (targets: the initial density and magnetic energy density of the
    seed-2 fields) with respect to the initial vector potential and velocity, n^3
    Mach-1 inputs (seed 1), `steps` FP64 steps, checkpoints every `ckpt` steps,
    each segment recomputed in the backward pass with its stage states recorded.
    Times: the plain forward (same steps, dt from eq. (cfl)), the checkpointing
    forward and the backward; the cost ratio is backward / plain forward."""
    import torch
    from paper_1812_04278_amd import binding, inputs, rollout
    f = inputs.random_fields(n, seed=1, v_rms=1.0, kmax=4)
    f2 = inputs.random_fields(n, seed=2, v_rms=1.0, kmax=4)
    p = binding.Patch(binding.config(n), device="cuda:0")
    p.init_from_potential(f2.rho, f2.v, f2.A, f2.P0, f2.B0)
    rho_t = p.hydro[0].clone()
    e_t = 0.5 * (p.bcell * p.bcell).sum(0)
    h3 = (1.0 / n) ** 3
    A0 = torch.as_tensor(f.A).to("cuda:0")
    v0 = torch.as_tensor(f.v).to("cuda:0")
    rho = torch.as_tensor(f.rho).to("cuda:0")

    def run():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p.init_from_potential(rho, v0, A0, f.P0, f.B0)
        for _ in range(steps):
            p.step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        A = A0.clone().requires_grad_(True)
        v = v0.clone().requires_grad_(True)
        hyd, bf, bc = rollout.rollout(A, v, rho, p, steps, ckpt_every=ckpt, P0=f.P0, B0=f.B0)
        J = h3 * (((hyd[0] - rho_t) ** 2).sum() + ((0.5 * (bc * bc).sum(0) - e_t) ** 2).sum())
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        gA, gv = torch.autograd.grad(J, [A, v])
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        return (t1 - t0) * 1e3, (t2 - t1) * 1e3, (t3 - t2) * 1e3, float(J.detach()), gA, gv

    run()                                           # warm-up (allocations, first launches)
    fwd, ck, bwd, J, gA, gv = run()
    return {"workload": f"{n}^3 periodic box, Mach 1, {steps} FP64 SSP-RK3 steps, checkpoints every {ckpt}, "
                        f"loss: L2 mismatch of final density and magnetic energy density vs a seed-2 target",
            "forward_ms": round(fwd, 2), "checkpointed_forward_ms": round(ck, 2), "backward_ms": round(bwd, 2),
            "ratio_backward_to_forward": round(bwd / fwd, 3), "ratio_total_to_forward": round((ck + bwd) / fwd, 3),
            "loss": J, "grad_norm_A": float(gA.norm()), "grad_norm_v": float(gv.norm())}


def mach5_512(steps: int = 10, ckpt: int = 2, n: int = 512):
    """The 512^3 workload: Mach 5 (v_rms 5, |k| <= 8), beta 0.5, the mixed form
    with an FP32 state (WM_MIXED_F32STATE), forward and adjoint in one run:
    throughput of `steps` steps with the update kernel's HBM rate, then the same
    steps as a checkpointed rollout (a checkpoint every `ckpt` steps, FP32) and
    its backward (the FP64 adjoint at the widened FP32 states, stage states
    recomputed by the FP32-state forward), timed against the plain forward.
    Inputs are generated on the GPU (same recipe and draws as the host
    generator)."""
    import math
    import torch
    from paper_1812_04278_amd import binding, inputs, rollout
    B0 = tuple(math.sqrt(2.4 / 1.25) * x for x in (1.0, 0.5, 0.0))
    log(f"bench {n}^3: generating inputs on the GPU")
    f = inputs.random_fields(n, seed=1, v_rms=5.0, kmax=8, B0=B0, device="cuda:0")
    rho, v0, A0 = f.rho, f.v, f.A
    out = {"workload": f"{n}^3 periodic box, Mach 5, |k| <= 8, beta 0.5, {steps} SSP-RK3 steps, FP32 state "
                       f"(mixed arithmetic), adjoint in FP64 at the widened states"}
    p = binding.Patch(binding.config(n, precision=binding.WM_MIXED_F32STATE), device="cuda:0")
    p.init_from_potential(rho, v0, A0, 0.6, B0)
    p.step()
    p.init_from_potential(rho, v0, A0, 0.6, B0)
    p.profile(True)
    ms = timed_steps(p, steps)
    rep = p.profile_report()
    p.profile(False)
    d = p.diagnostics(raise_unphysical=False)
    nup, msup = rep["update"]
    upd_ms = msup / max(nup, 1)
    upd_bytes = UPDATE_VALUES_PER_ZONE * 4 * float(n) ** 3
    sw_ms = rep["sweep"][1] / max(rep["sweep"][0], 1)
    sw_tf = FLOPS_PER_FACE * float(n) ** 3 / (sw_ms * 1e-3) / 1e12
    out["f32state"] = {"value": round(n ** 3 * steps / (ms * 1e-3) / 1e6, 3), "unit": "Mzone-updates/s",
                       "ms_per_step": round(ms / steps, 3),
                       "sweep_avg_ms": round(sw_ms, 4), "sweep_tflops": round(sw_tf, 3),
                       # FP32 vector instructions issue at the FP64 rate with packed FP32 off
                       "sweep_frac_fp64_vector_peak": round(sw_tf / PEAK_FP64_TFLOPS, 4),
                       "update_avg_ms": round(upd_ms, 4),
                       "update_hbm_gbs": round(upd_bytes / (upd_ms * 1e-3) / 1e9, 1),
                       "update_hbm_frac": round(upd_bytes / (upd_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                       "max_divb": d["max_divb"], "n_unphysical": d["n_unphysical"], "min_p": d["min_p"]}
    log("bench 512^3: checkpointed FP32-state rollout and its adjoint")
    A = A0.clone().requires_grad_(True)
    v = v0.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    hyd, bf, bc = rollout.rollout(A, v, rho, p, steps, ckpt_every=ckpt, P0=0.6, B0=B0, store_stages=False)
    J = (1.0 / n) ** 3 * ((hyd[0].double() - 1.0) ** 2).sum()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    gA, gv = torch.autograd.grad(J, [A, v])
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    ck_ms, bwd_ms = (t2 - t1) * 1e3, (t3 - t2) * 1e3
    out["adjoint"] = {"forward_ms": round(ms, 1), "checkpointed_forward_ms": round(ck_ms, 1),
                      "backward_ms": round(bwd_ms, 1), "ratio_backward_to_forward": round(bwd_ms / ms, 3),
                      "ratio_total_to_forward": round((ck_ms + bwd_ms) / ms, 3),
                      "loss": "h^3 sum (rho_T - 1)^2", "stage_states": "recomputed", "ckpt_every": ckpt,
                      "grad_finite": bool(torch.isfinite(gA).all() and torch.isfinite(gv).all()),
                      "peak_gib": round(torch.cuda.max_memory_allocated() / 2 ** 30, 1)}
    del p, gA, gv, A, v, hyd, bf, bc, J
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--cpu-threads", type=int, default=0, help="oracle threads (0: torch's default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the FP64-vs-mixed comparison")
    ap.add_argument("--no-convergence", action="store_true", help="skip the fast-wave convergence table")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint cost measurement")
    ap.add_argument("--no-rk4", action="store_true", help="skip the RK4 (CFL 0.8) throughput leg")
    ap.add_argument("--no-waves", action="store_true", help="skip the oblique linear-wave suite")
    ap.add_argument("--wave-sizes", default="16,32,64", help="N of the 2N x N x N wave boxes")
    ap.add_argument("--wave-weights", default="z", choices=("z", "z_printed", "js"),
                    help="WENO weights of the wave suite: WENO-Z (reading), WENO-Z as printed, Jiang-Shu")
    ap.add_argument("--no-512", action="store_true",
                    help="skip the 512^3 Mach-5 workload (FP32-state forward and its adjoint)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU: the library has no multi-GPU brick decomposition "
              "(halo exchange and dt all-reduce are not implemented); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1812_04278_amd import binding, inputs

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    n = args.n
    log(f"bench: generating {n}^3 Mach-2 inputs")
    f = inputs.random_fields(n, seed=1, v_rms=2.0, kmax=4)
    p = binding.Patch(binding.config(n), device="cuda:0")
    p.init_from_potential(f.rho, f.v, f.A, f.P0, f.B0)
    log(f"bench: warmup {args.warmup} step(s)")
    for _ in range(args.warmup):
        p.step()
    torch.cuda.synchronize()
    # timed run restarts from the initial state: steps 1..K of the workload
    p.init_from_potential(f.rho, f.v, f.A, f.P0, f.B0)
    torch.cuda.synchronize()
    p.profile(True)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(p.stream)
    for s in range(args.steps):
        p.step()
    ev1.record(p.stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    gpu_ms = ev0.elapsed_time(ev1)
    rep = p.profile_report()
    p.profile(False)
    d = p.diagnostics(raise_unphysical=False)
    log(f"bench: {args.steps} steps in {wall * 1e3:.1f} ms (events {gpu_ms:.1f} ms); kernels {rep}")

    ms_step = wall * 1e3 / args.steps
    value = n ** 3 * args.steps / wall / 1e6
    nsw, msw = rep["sweep"]
    sweep_ms = msw / max(nsw, 1)
    flops = FLOPS_PER_FACE * float(n) ** 3
    ach = flops / (sweep_ms * 1e-3) / 1e12
    nup, msup = rep["update"]
    upd_ms = msup / max(nup, 1)
    # update kernel, algorithmic bytes per zone averaged over the three stages:
    # reads 21 face values + 8 U^n + 8 acc (stages 1, 2); writes 8 state + 8 acc (stages 0, 1)
    upd_bytes = UPDATE_VALUES_PER_ZONE * 8 * float(n) ** 3
    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "Mzone-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{n}^3 periodic MHD box, Mach 2, beta~1, WENO5-JS + CT, SSP-RK3 CFL 0.4, FP64",
                   "grid": n, "steps": args.steps, "precision": "fp64", "seed": 1},
        "roofline": {"kernel": "sweep", "bound": "alu", "achieved": round(ach, 3), "peak": PEAK_FP64_TFLOPS,
                     "unit": "TFLOP/s", "frac": round(ach / PEAK_FP64_TFLOPS, 4),
                     "traffic": SWEEP_TRAFFIC_BYTES_256 if n == 256 else None,
                     "avg_ms": round(sweep_ms, 4), "launches": nsw, "flops_per_launch": flops},
        "roofline_update": {"kernel": "update", "bound": "hbm",
                            "achieved": round(upd_bytes / (upd_ms * 1e-3) / 1e9, 1), "peak": PEAK_HBM_GBS,
                            "unit": "GB/s", "frac": round(upd_bytes / (upd_ms * 1e-3) / 1e9 / PEAK_HBM_GBS, 4),
                            "avg_ms": round(upd_ms, 4)},
        "kernel_ms_per_step": {k: round(v[1] / args.steps, 4) for k, v in rep.items()},
        "diagnostics_after": {"max_divb": d["max_divb"], "n_unphysical": d["n_unphysical"]},
        "context": "paper: ~0.6 Mzone/s per 36-core Broadwell node (FP64, RK4, with MPI)",
    }
    if not args.no_mixed:
        log("bench: mixed precision vs FP64 (Mach 0.1 workload)")
        out["mixed"] = mixed_precision(n, args.steps)
    if not args.no_rk4:
        log("bench: classical RK4 at CFL 0.8 vs SSP-RK3 at CFL 0.4")
        out["rk4"] = rk4_leg(n, args.steps)
    if not args.no_waves:
        log("bench: oblique linear waves (WENO-Z, RK4 at CFL 0.8)")
        out["oblique_waves"] = oblique_waves(tuple(int(x) for x in args.wave_sizes.split(",")),
                                              weights=args.wave_weights)
    if not args.no_convergence:
        log("bench: fast-wave convergence, both precisions")
        out["convergence"] = convergence((32, 64, 128, 256))
    if not args.no_adjoint:
        log("bench: adjoint cost (128^3, 20 steps, checkpoints every 5)")
        out["adjoint"] = adjoint_cost()
    if not args.no_512:
        log("bench: 512^3 Mach-5 workload, FP32 state, forward and adjoint")
        out["mach5_512"] = mach5_512()
    if args.copy_calibration:
        # a plain copy of known size: 1 GiB read + 1 GiB written, for scaling
        # the FETCH_SIZE / WRITE_SIZE counters of the kernels above
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = src.numel() * 8
        del src, dst
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle: 32^3 x 1 and 64^3 x 10 on all threads, then one thread)")
        out["cpu_baseline"] = cpu_baseline(args.cpu_threads or None)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
