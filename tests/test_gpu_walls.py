"""Reflecting conducting walls and floors on the GPU against the oracle
(readings R20, R21).  Boxes span several tiles along the walled axis with
ragged tails (a walled axis also computes the lower wall face, which shifts the
tiles by one), and the all-walls box has an x axis (22 zones) shorter than the
x tile (64 faces), whose stencil positions run past the mirror-doubled axis.
Bars: FP64 <= 1e-12 normwise relative per variable; the normal field on the
wall faces exactly zero; floor activations counted equally; mixed forms one
step <= 5e-8 (FP64 state, v_rms 0.8) and <= 1e-6 (FP32 state)."""
import dataclasses
import sys

import pytest
import torch

from oracle import mhd
from paper_1812_04278_amd import binding as B
from helpers import assert_state_parity, rel_err, state_errors, walled_state

pytestmark = pytest.mark.gpu

CASES = [((70, 20, 18), (True, False, False)), ((21, 40, 18), (False, True, False)),
         ((20, 18, 35), (False, False, True)), ((22, 19, 20), (True, True, True)),
         # the walled axes' faces (zones + the lower wall face) exactly fill one tile:
         # x 63 + 1 = 64 (x tile), y 31 + 1 = 32 (FP64 y tile)
         ((63, 31, 12), (True, True, False))]


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.load()


def gpu_patch(U, cfg, **kw):
    p = B.Patch(B.config(nx=cfg.nx, ny=cfg.ny, nz=cfg.nz, h=cfg.h, walls=tuple(int(w) for w in cfg.walls),
                         rho_floor=cfg.rho_floor, p_floor=cfg.p_floor, **kw))
    p.set_state(U["rho"], U["m"], U["E"], U["b"])
    return p


def oracle_sweep_walled(U, axis, cfg):
    """The oracle's sweep on the mirror-doubled box, cropped to the box."""
    D, n = U, [cfg.nx, cfg.ny, cfg.nz]
    for w in range(3):
        if cfg.walls[w]:
            D = mhd.mirror_double(D, w)
    sizes = [n[w] * (2 if cfg.walls[w] else 1) for w in range(3)]
    cfgD = dataclasses.replace(cfg, nx=sizes[0], ny=sizes[1], nz=sizes[2], walls=(False, False, False))
    F, T = mhd.sweep(D, axis, cfgD)
    for w in range(3):
        if cfg.walls[w]:
            F = F.narrow(2 - w, 0, n[w])
            T = T.narrow(3 - w, 0, n[w])
    return F, T


@pytest.mark.parametrize("shape,walls", CASES)
def test_walled_sweeps_and_rhs(shape, walls):
    say(f"walled sweeps and rhs {shape} walls {walls}")
    U, cfg = walled_state(n=shape, walls=walls)
    p = gpu_patch(U, cfg)
    for axis in range(3):
        out = p.debug_sweep(axis).cpu()
        F, T = oracle_sweep_walled(U, axis, cfg)
        for c in range(7):
            assert rel_err(out[c], F[..., c]) <= 1e-12, (axis, c)
        for c in range(2):
            assert rel_err(out[7 + c], T[c]) <= 1e-12, (axis, "T", c)
    k = p.debug_rhs().cpu()
    ko = mhd.rhs(U, cfg)
    ref = [ko["rho"], ko["m"][0], ko["m"][1], ko["m"][2], ko["E"], ko["b"][0], ko["b"][1], ko["b"][2]]
    for c in range(8):
        assert rel_err(k[c], ref[c]) <= 1e-12, ("rhs", c, rel_err(k[c], ref[c]))


@pytest.mark.parametrize("weights", [B.WM_WENO_JS, B.WM_WENO_Z])
def test_walled_rk4_steps(weights):
    """The paper's RK4 at CFL 0.8 (reading R16) on the all-walls box, with both
    weight families: two steps against the oracle's RK4 at the same dt."""
    say(f"walled RK4 steps 22x19x20, weights {weights}")
    U, cfg = walled_state(n=(22, 19, 20), walls=(True, True, True))
    wz = weights == B.WM_WENO_Z
    if wz:
        cfg = dataclasses.replace(cfg, weights="z")
    p = gpu_patch(U, cfg, integrator=B.WM_RK4, cfl=0.8, weights=weights)
    dt = mhd.compute_dt(U, dataclasses.replace(cfg, cfl=0.8))
    for _ in range(2):
        p.step_dt(dt)
        U, _ = mhd.step_rk4(U, cfg, dt)
    assert_state_parity(p.state(), U, label=f"walled RK4 weights {weights}")


@pytest.mark.parametrize("shape,walls", CASES)
def test_walled_steps(shape, walls):
    """Three steps (dt from each side's eq. cfl): parity, the wall faces' normal
    field exactly zero, mass and energy conserved to round-off."""
    say(f"walled steps {shape} walls {walls}")
    U, cfg = walled_state(n=shape, walls=walls)
    p = gpu_patch(U, cfg)
    d0 = p.diagnostics()
    for _ in range(3):
        dt_g = p.step(want_dt=True)
        U, dt_o = mhd.step(U, cfg)
        assert abs(dt_g - dt_o) <= 1e-13 * dt_o
    g = p.state()
    assert_state_parity(g, U, label=f"walls {walls}")
    n = [cfg.nx, cfg.ny, cfg.nz]
    for axis in range(3):
        if walls[axis]:
            assert float(g["b"][axis].narrow(2 - axis, n[axis] - 1, 1).abs().max()) == 0.0
    d1 = p.diagnostics()
    assert abs(d1["mass"] - d0["mass"]) <= 1e-13 * abs(d0["mass"])
    assert abs(d1["energy"] - d0["energy"]) <= 1e-13 * abs(d0["energy"])
    assert d1["max_divb"] <= 1e-12 / cfg.h


def test_walled_init_from_potential():
    """init_from_potential on a walled box zeroes the wall faces and matches the
    oracle's initial state (walls-aware zone field in the energy)."""
    say("walled init 22x19x20")
    from paper_1812_04278_amd import inputs
    U, cfg = walled_state(n=(22, 19, 20), walls=(True, False, True))
    f = inputs.random_fields(22, 3, 0.8, kmax=2, B0=(0.0, 0.0, 0.0))
    rho = f.rho[:20, :19, :22].copy()
    v = f.v[:, :20, :19, :22].copy()
    A = f.A[:, :20, :19, :22].copy()
    B0 = (0.0, 0.6, 0.0)
    Uo = mhd.init_from_potential(rho, v, A, f.P0, B0, cfg)
    p = B.Patch(B.config(nx=22, ny=19, nz=20, h=cfg.h, walls=(1, 0, 1)))
    p.init_from_potential(rho, v, A, f.P0, B0)
    assert_state_parity(p.state(), Uo, label="walled init")
    assert rel_err(p.bcell.cpu(), mhd.zone_B_cfg(Uo["b"], cfg)) <= 1e-12


@pytest.mark.parametrize("shape,walls", [((70, 20, 18), (True, False, False)), ((22, 19, 20), (True, True, True)),
                                         ((21, 40, 18), (False, True, False))])
@pytest.mark.parametrize("precision,tol", [(B.WM_MIXED, 5e-8), (B.WM_MIXED_F32STATE, 1e-6)])
def test_walled_step_mixed(precision, tol, shape, walls):
    """One mixed step of a walled box.  The walled state moves at v_rms = 0.8,
    not Mach 0.1: the mixed error grows with the flux corrections carried in
    FP32 (periodic one step at Mach 0.1: 1.8e-9; ten steps at Mach 2: 4.7e-8),
    so the bar is the Mach-2 one, 5e-8 (measured 1.4e-8); FP32 state 1e-6.
    The FP32-state update takes two x-adjacent zones per thread when nx is
    even (70, 22) and one otherwise (21)."""
    say(f"walled step {shape} walls {walls}, precision {precision}")
    U, cfg = walled_state(n=shape, walls=walls)
    p = gpu_patch(U, cfg, precision=precision)
    dt = mhd.compute_dt(U, cfg)
    p.step_dt(dt)
    U1, _ = mhd.step(U, cfg, dt)
    errs = state_errors(p.state(), U1)
    say("  ", {k: f"{v:.2e}" for k, v in errs.items()})
    assert max(errs.values()) <= tol, errs


def test_floors_parity_and_counts():
    """Floors above the state's minima: the activations of two steps counted
    equally on both sides and the states agree (FP64)."""
    say("floors 24x20x16 walls x")
    U, cfg = walled_state(n=(24, 20, 16), walls=(True, False, False))
    rho_min = float(U["rho"].min())
    _, _, _, P = mhd.primitives(U, cfg.gamma, cfg)
    cfg = dataclasses.replace(cfg, rho_floor=rho_min + 0.02, p_floor=float(P.min()) + 0.01)
    p = gpu_patch(U, cfg)
    stats = {}
    for _ in range(2):
        U, dt = mhd.step(U, cfg, None, stats)
        p.step_dt(dt)
    d = p.diagnostics()
    say(f"  floor activations: gpu {d['n_floored']} oracle {stats['n_floored']}")
    assert stats["n_floored"] > 0 and d["n_floored"] == stats["n_floored"]
    assert_state_parity(p.state(), U, label="floors")
    # rebinding the state restarts the count
    p.set_state(U["rho"], U["m"], U["E"], U["b"])
    assert p.diagnostics()["n_floored"] == 0


@pytest.mark.parametrize("kw", [dict(walls=(True, False, False)), dict(rho_floor=1e-3)])
def test_adjoint_refuses_walls_and_floors(kw):
    """The adjoint covers periodic boxes without floors (walls and floors are
    not differentiated): its calls refuse such a patch with WM_ERR_ARG before
    any launch."""
    say(f"adjoint refusal {kw}")
    walls = kw.get("walls", (False, False, False))
    U, cfg = walled_state(n=(12, 10, 8), walls=walls)
    cfg = dataclasses.replace(cfg, rho_floor=kw.get("rho_floor", 0.0))
    p = gpu_patch(U, cfg)
    lam = torch.zeros((8, cfg.nz, cfg.ny, cfg.nx), dtype=torch.float64, device="cuda")
    with pytest.raises(B.WmError) as e:
        p.rhs_vjp(p.hydro, p.bface, lam)
    assert e.value.status == B.WM_ERR_ARG
    with pytest.raises(B.WmError) as e:
        p.adjoint_step(p.hydro.clone(), p.bface.clone(), 1e-3, lam[:5].clone(), lam[5:].clone())
    assert e.value.status == B.WM_ERR_ARG
