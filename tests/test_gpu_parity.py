"""GPU parity: the HIP path through the C ABI against the FP64 oracle on the same
seeded inputs.  Bar: normwise relative difference per variable <= 1e-12
(max_i |gpu_i - oracle_i| / max_i |oracle_i|), FP64."""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import mhd
from paper_1812_04278_amd import binding as B
from helpers import T64, _subbox, assert_diag_parity, assert_state_parity, diag_state, fields, oracle_state, rel_err

pytestmark = pytest.mark.gpu
TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_patch(f, **kw):
    nz, ny, nx = f.rho.shape
    p = B.Patch(B.config(nx=nx, ny=ny, nz=nz, h=1.0 / nx, **kw))
    p.init_from_potential(f.rho, f.v, f.A, f.P0, f.B0)
    return p


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    B.load()


def test_init_parity():
    say("init parity 37x21x19")
    f = fields(40, seed=3, v_rms=1.0, crop=(37, 21, 19))
    U, cfg = oracle_state(f)
    p = gpu_patch(f)
    assert_state_parity(p.state(), U, label="init")
    assert rel_err(p.bcell.cpu(), mhd.zone_B(U["b"])) <= TOL


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_sweep_parity(axis):
    """Interface fluxes (7 sweep-frame components) and CT transport fluxes of one
    sweep, on a box that spans several tiles with ragged tails in every direction."""
    say(f"sweep parity axis {axis}")
    f = fields(40, seed=4, v_rms=1.5, crop=(37, 21, 19))
    U, cfg = oracle_state(f)
    p = gpu_patch(f)
    out = p.debug_sweep(axis).cpu()
    F, T = mhd.sweep(U, axis, cfg)
    for c in range(7):
        e = rel_err(out[c], F[..., c])
        assert e <= TOL, (axis, c, e)
    for c in range(2):
        e = rel_err(out[7 + c], T[c])
        assert e <= TOL, (axis, "T", c, e)


def test_rhs_parity():
    say("rhs parity 37x21x19")
    f = fields(40, seed=5, v_rms=1.5, crop=(37, 21, 19))
    U, cfg = oracle_state(f)
    p = gpu_patch(f)
    k = p.debug_rhs().cpu()
    ko = mhd.rhs(U, cfg)
    ref = [ko["rho"], ko["m"][0], ko["m"][1], ko["m"][2], ko["E"], ko["b"][0], ko["b"][1], ko["b"][2]]
    for c in range(8):
        e = rel_err(k[c], ref[c])
        assert e <= TOL, (c, e)


def test_step_32_mach01():
    """One SSP-RK3 step on 32^3, Mach 0.1 (the small FP64 workload), dt from
    eq. (cfl) on each side."""
    say("step 32^3")
    f = fields(32, seed=1, v_rms=0.1)
    U, cfg = oracle_state(f)
    p = gpu_patch(f)
    dt_g = p.step(want_dt=True)
    U1, dt_o = mhd.step(U, cfg)
    assert abs(dt_g - dt_o) <= 1e-14 * dt_o
    assert_state_parity(p.state(), U1, label="step")
    assert rel_err(p.bcell.cpu(), mhd.zone_B(U1["b"])) <= TOL


def test_stages_with_given_dt():
    say("stages with host dt 24x20x28")
    f = fields(32, seed=6, v_rms=1.0, crop=(24, 20, 28))
    U, cfg = oracle_state(f)
    p = gpu_patch(f)
    dt = 0.3 * mhd.compute_dt(U, cfg)
    for s in range(3):
        p.rk_stage(s, dt)
    U1, _ = mhd.step(U, cfg, dt)
    assert_state_parity(p.state(), U1, label="stages")


@pytest.mark.parametrize("n", [4, 5, 8])
def test_tiny_grids(n):
    """Brute force on tiny grids (every stage, two steps): the periodic wrap of the
    6-zone stencil covers the whole box several times."""
    say(f"tiny grid {n}")
    f = fields(n, seed=7 + n, v_rms=0.5, kmax=1)
    U, cfg = oracle_state(f)
    p = gpu_patch(f)
    for _ in range(2):
        dt_g = p.step(want_dt=True)
        U, dt_o = mhd.step(U, cfg)
        assert abs(dt_g - dt_o) <= 1e-14 * dt_o
    assert_state_parity(p.state(), U, label=f"tiny {n}")


def test_crop_64_ten_steps_mach2():
    """The 256^3 Mach-2 workload's generator sampled at 64^3, 10 steps, full-field
    parity against the oracle (dt from each side's own eq. (cfl))."""
    say("64^3 Mach 2, 10 steps")
    f = fields(64, seed=1, v_rms=2.0)
    U, cfg = oracle_state(f)
    p = gpu_patch(f)
    for s in range(10):
        dt_g = p.step(want_dt=True)
        U, dt_o = mhd.step(U, cfg)
        assert abs(dt_g - dt_o) <= 1e-13 * dt_o, (s, dt_g, dt_o)
        say(f"  step {s} dt {dt_g:.6e}")
    assert_state_parity(p.state(), U, label="64^3 x 10")
    # diagnostics of the oracle's state, loaded into the patch (same state on both sides)
    p.set_state(U["rho"], U["m"], U["E"], U["b"])
    assert_diag_parity(p.diagnostics(), mhd.diagnostics(U, cfg), U, cfg.h)


WZ_FORMS = [("z", B.WM_WENO_Z), ("z_printed", B.WM_WENO_Z_PRINTED)]


@pytest.mark.parametrize("form,wcode", WZ_FORMS)
def test_wenoz_step_32_mach01(form, wcode):
    """WENO-Z weights (reading R13, and the form Sect. 2.2 prints): one step on
    32^3, Mach 0.1, dt from eq. (cfl)."""
    import dataclasses
    say(f"WENO-Z ({form}) step 32^3")
    f = fields(32, seed=1, v_rms=0.1)
    U, cfg = oracle_state(f)
    cfg = dataclasses.replace(cfg, weights=form)
    p = gpu_patch(f, weights=wcode)
    dt_g = p.step(want_dt=True)
    U1, dt_o = mhd.step(U, cfg)
    assert abs(dt_g - dt_o) <= 1e-14 * dt_o
    assert_state_parity(p.state(), U1, label=f"WENO-Z ({form}) step")


@pytest.mark.parametrize("form,wcode", WZ_FORMS)
def test_wenoz_ten_steps_64_mach2_ragged(form, wcode):
    """WENO-Z over ten Mach-2 steps on a ragged 40 x 36 x 34 crop of the 64^3
    generator (shocks start to form), dt from the oracle each step."""
    import dataclasses
    say(f"WENO-Z ({form}) 10 steps 40x36x34 Mach 2")
    f = fields(64, seed=1, v_rms=2.0, crop=(40, 36, 34))
    U, cfg = oracle_state(f, h=1.0 / 64)
    cfg = dataclasses.replace(cfg, weights=form)
    nz, ny, nx = U["rho"].shape
    p = B.Patch(B.config(nx=nx, ny=ny, nz=nz, h=1.0 / 64, weights=wcode))
    p.set_state(U["rho"], U["m"], U["E"], U["b"])
    for _ in range(10):
        U, dt = mhd.step(U, cfg)
        p.step_dt(dt)
    assert_state_parity(p.state(), U, label=f"WENO-Z ({form}) 10 steps")


def test_uniform_state_bitwise():
    say("uniform state")
    n = 20
    ones = np.ones((n, n, n))
    v = np.stack([0.7 * ones, -0.4 * ones, 0.25 * ones])
    p = B.Patch(B.config(n))
    p.init_from_potential(1.3 * ones, v, np.zeros((3, n, n, n)), 0.6, (1.0, 0.5, -0.3))
    h0, b0 = p.hydro.clone(), p.bface.clone()
    for _ in range(3):
        p.step()
    torch.cuda.synchronize()
    assert torch.equal(p.hydro, h0) and torch.equal(p.bface, b0)


def test_determinism():
    say("determinism")
    f = fields(48, seed=8, v_rms=2.0)
    outs = []
    for _ in range(2):
        p = gpu_patch(f)
        for _ in range(3):
            p.step()
        torch.cuda.synchronize()
        outs.append((p.hydro.clone(), p.bface.clone()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


@pytest.mark.parametrize("precision,walls", [(B.WM_FP64, (0, 0, 0)), (B.WM_FP64, (1, 0, 1)),
                                             (B.WM_MIXED_F32STATE, (0, 0, 0))])
def test_wide_addressing_bitwise(precision, walls):
    """The sweep's 64-bit addressing path, which it takes for arrays of 4 GiB or
    more, gives bitwise the same steps as its 32-bit buffer-offset path."""
    say(f"wide addressing, precision {precision}, walls {walls}")
    f = fields(40, seed=9, v_rms=2.0)
    outs = []
    for wide in (False, True):
        p = gpu_patch(f, precision=precision, walls=walls)
        p.debug_wide_addressing(wide)
        for _ in range(2):
            p.step()
        torch.cuda.synchronize()
        outs.append((p.hydro.clone(), p.bface.clone()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][1], outs[1][1])


def test_invariants_128_mach2():
    """Conservation of totals and plane sums and div_h b at round-off, 128^3 x 5 steps."""
    say("invariants 128^3")
    f = fields(128, seed=1, v_rms=2.0)
    p = gpu_patch(f)
    d0 = p.diagnostics()
    planes = ((0, (0, 1)), (1, (0, 2)), (2, (1, 2)))
    s0 = [p.bface[c].sum(dim=d).cpu() for c, d in planes]
    scale = [float(p.bface[c].abs().sum(dim=d).max()) for c, d in planes]   # sum of |b| over a plane
    for _ in range(5):
        p.step()
    d1 = p.diagnostics()
    assert d1["n_unphysical"] == 0
    assert abs(d1["mass"] - d0["mass"]) <= 1e-13 * abs(d0["mass"])
    assert abs(d1["energy"] - d0["energy"]) <= 1e-13 * abs(d0["energy"])
    for c in range(3):
        assert abs(d1["mom"][c] - d0["mom"][c]) <= 1e-13 * (abs(d0["mass"]) * 2.0)
    s1 = [p.bface[c].sum(dim=d).cpu() for c, d in planes]
    for a, b, sc in zip(s0, s1, scale):
        assert float((a - b).abs().max()) <= 1e-13 * sc
    h = 1.0 / 128
    assert d1["max_divb"] <= 1e-12 / h


def test_full_size_sampled_256():
    """The 256^3 Mach-2 workload in the launch configuration the benchmark times:
    the GPU right-hand side and one GPU step, checked at sampled zones against the
    oracle run on a periodic sub-box around each sample (the step's dependence
    radius is below the sub-box margin: 6 zones per stage)."""
    say("256^3 sampled parity")
    f = fields(256, seed=1, v_rms=2.0)
    p = gpu_patch(f)
    st0 = p.state()
    k = p.debug_rhs().cpu()
    dt = p.compute_dt()
    # dt against the oracle's eq. (cfl) on the full box (cheap reduction)
    cfg_full = mhd.cubic(256)
    dt_o = mhd.compute_dt(st0, cfg_full)
    assert abs(dt - dt_o) <= 1e-14 * dt_o
    p.step()
    st1 = p.state()
    g = torch.Generator().manual_seed(11)
    cents = [tuple(int(x) for x in torch.randint(0, 256, (3,), generator=g)) for _ in range(3)]
    cfg16 = mhd.Config(16, 16, 16, 1.0 / 256)
    cfg48 = mhd.Config(48, 48, 48, 1.0 / 256)
    for c in cents:
        sub = {key: _subbox(st0[key], c, 8) for key in st0}
        ko = mhd.rhs(sub, cfg16)
        ref = [ko["rho"], ko["m"][0], ko["m"][1], ko["m"][2], ko["E"], ko["b"][0], ko["b"][1], ko["b"][2]]
        for comp in range(8):
            gv = float(_subbox(k[comp], c, 8)[8, 8, 8])
            ov = float(ref[comp][8, 8, 8])
            scale = float(ref[comp].abs().max())
            assert abs(gv - ov) <= TOL * scale, (c, comp, gv, ov)
        sub = {key: _subbox(st0[key], c, 24) for key in st0}
        U1, _ = mhd.step(sub, cfg48, dt)
        for key in ("rho", "E"):
            gv = _subbox(st1[key], c, 24)[20:28, 20:28, 20:28]
            ov = U1[key][20:28, 20:28, 20:28]
            assert rel_err(gv, ov) <= TOL, (c, key)
        for key in ("m", "b"):
            gv = _subbox(st1[key], c, 24)[:, 20:28, 20:28, 20:28]
            ov = U1[key][:, 20:28, 20:28, 20:28]
            for comp in range(3):
                assert rel_err(gv[comp], ov[comp]) <= TOL, (c, key, comp)
        say(f"  sample {c} ok")


FUSED_DT_CASES = [
    ("fp64", (37, 21, 19), dict()),
    ("mixed", (37, 21, 19), dict(precision=B.WM_MIXED)),
    ("f32state", (37, 21, 19), dict(precision=B.WM_MIXED_F32STATE)),
    ("rk4-wenoz", (33, 24, 20), dict(integrator=B.WM_RK4, weights=B.WM_WENO_Z)),
    ("walls", (22, 19, 20), dict(walls=(1, 0, 1))),
    ("tiny", (3, 2, 5), dict(precision=B.WM_MIXED_F32STATE)),
    # the per-wave maxima do not fit the FP32 accumulator: the step takes the stand-alone pass
    ("thin-f32", (1, 1, 16), dict(precision=B.WM_MIXED_F32STATE)),
]


@pytest.mark.parametrize("name,shape,kw", FUSED_DT_CASES, ids=[c[0] for c in FUSED_DT_CASES])
def test_fused_dt_bitwise(name, shape, kw):
    """A step takes the maxima of eq. (cfl) from its first stage's sweeps: its
    dt, and the state after it, are bitwise those of the stand-alone time-step
    pass (wm_compute_dt) followed by the stages with that dt, over three steps,
    for every precision mode, RK4 with WENO-Z weights, walls, a box smaller than
    one tile in every direction, and a 1 x 1 x 16 FP32-state box, whose step falls
    back to the stand-alone pass."""
    say(f"fused dt {name} {shape}")
    nx, ny, nz = shape
    f = fields(max(shape), seed=12, v_rms=1.0, crop=shape)
    a = gpu_patch(f, **kw)
    b = gpu_patch(f, **kw)
    for n in range(3):
        dt_b = b.compute_dt()
        b.step_dt(dt_b)
        dt_a = a.step(want_dt=True)
        assert math.isfinite(dt_a) and dt_a > 0.0
        assert dt_a == dt_b, (name, n, dt_a, dt_b)
        sa, sb = a.state(), b.state()
        for k in ("rho", "m", "E", "b"):
            assert torch.equal(sa[k], sb[k]), (name, n, k)
    say(f"  dt {dt_a:.17g} ok")


@pytest.mark.parametrize("damage", ["zero_energy", "nan_density", "infinite_energy"])
def test_fused_dt_damaged_state(damage):
    """The failure semantics of the fused time step match the stand-alone pass:
    a zone with E = 0 (negative gas pressure), a NaN density, or an infinite
    energy gives a step whose dt is bitwise that of wm_compute_dt, or NaN on
    both sides (a NaN density always gives NaN)."""
    say(f"fused dt, damaged state: {damage}")
    f = fields(16, seed=3, v_rms=0.3, kmax=2)
    pa, pb = gpu_patch(f), gpu_patch(f)
    st = pa.state()
    rho, E = st["rho"].clone(), st["E"].clone()
    if damage == "zero_energy":
        E[3, 4, 5] = 0.0
    elif damage == "nan_density":
        rho[7, 8, 9] = float("nan")
    else:
        E[2, 2, 2] = float("inf")
    for p in (pa, pb):
        p.set_state(rho, st["m"], E, st["b"])
    dt_b = pb.compute_dt()
    dt_a = pa.step(want_dt=True)
    if damage == "nan_density":
        assert math.isnan(dt_a) and math.isnan(dt_b)
    else:
        assert dt_a == dt_b or (math.isnan(dt_a) and math.isnan(dt_b)), (dt_a, dt_b)
    say(f"  dt step {dt_a!r}, stand-alone {dt_b!r}")


def test_failure_injection_unphysical():
    """Host-side failure injection: a zone with E = 0 (negative gas pressure) and a
    zone with a NaN density are reported by the diagnostics -- WM_ERR_UNPHYSICAL
    with n_unphysical = 2 and the negative minimum pressure -- and a step from
    that state still runs to completion, with a non-finite dt (the maxima of
    eq. (cfl) propagate NaN) and the damage flagged afterwards."""
    say("failure injection 16^3")
    f = fields(16, seed=3, v_rms=0.3, kmax=2)
    p = gpu_patch(f)
    st = p.state()
    rho, E = st["rho"].clone(), st["E"].clone()
    E[3, 4, 5] = 0.0
    rho[7, 8, 9] = float("nan")
    p.set_state(rho, st["m"], E, st["b"])
    with pytest.raises(B.WmError) as e:
        p.diagnostics()
    assert e.value.status == B.WM_ERR_UNPHYSICAL
    d = p.diagnostics(raise_unphysical=False)
    assert d["n_unphysical"] == 2, d
    assert d["min_p"] < 0.0
    Ub = dict(rho=rho, m=st["m"], E=E, b=st["b"])
    assert_diag_parity(d, mhd.diagnostics(Ub, mhd.cubic(16)), Ub, 1.0 / 16)
    dt = p.step(want_dt=True)
    assert not math.isfinite(dt)
    assert p.diagnostics(raise_unphysical=False)["n_unphysical"] >= 2


def test_side_stream_matches_default():
    """A patch created on its own stream (default priority) gives bitwise the
    state of a patch on the current stream: initial state, three steps, the
    host copy, and set_state round trips, with the caller's stream left busy."""
    say("side stream 24x20x16")
    f = fields(24, seed=5, v_rms=1.0, crop=(24, 20, 16))
    ref = gpu_patch(f)
    for _ in range(3):
        ref.step()
    r = ref.state()
    side = torch.cuda.Stream()
    nz, ny, nx = f.rho.shape
    p = B.Patch(B.config(nx=nx, ny=ny, nz=nz, h=1.0 / nx), stream=side)
    busy = torch.randn(4096, 4096, device="cuda", dtype=torch.float64)
    for _ in range(4):
        busy = busy @ busy * 1e-3           # keep the caller's stream occupied
    p.init_from_potential(f.rho, f.v, f.A, f.P0, f.B0)
    st0 = p.state()
    p.set_state(st0["rho"], st0["m"], st0["E"], st0["b"])
    for _ in range(3):
        p.step()
    g = p.state()
    for k in ("rho", "m", "E", "b"):
        assert torch.equal(g[k], r[k]), k
    torch.cuda.synchronize()


@pytest.mark.parametrize("shape", [(24, 20, 1), (32, 1, 1), (1, 12, 10), (1, 1, 1)])
def test_degenerate_dimensions(shape):
    """Boxes one zone thick: nz = 1 is the 2D scheme, ny = nz = 1 the 1D one (the
    sweep along a one-zone direction sees a uniform stencil and adds no flux
    difference); 1 x 1 x 1 leaves the state exactly unchanged.  Three steps
    against the oracle, dt from each side's eq. (cfl)."""
    nx, ny, nz = shape
    say(f"degenerate box {shape}")
    f = fields(max(shape + (8,)), seed=9, v_rms=1.0, kmax=2, crop=shape)
    U, cfg = oracle_state(f, h=1.0 / max(shape))
    p = B.Patch(B.config(nx=nx, ny=ny, nz=nz, h=cfg.h))
    p.init_from_potential(f.rho, f.v, f.A, f.P0, f.B0)
    assert_state_parity(p.state(), U, label=f"{shape} init")
    U0 = {k: v.clone() for k, v in U.items()}
    for _ in range(3):
        dt_g = p.step(want_dt=True)
        U, dt_o = mhd.step(U, cfg)
        assert abs(dt_g - dt_o) <= 1e-14 * dt_o
    assert_state_parity(p.state(), U, label=f"{shape} 3 steps")
    if shape == (1, 1, 1):
        g = p.state()
        for k in U0:
            assert torch.equal(g[k], U0[k]), k


@pytest.mark.parametrize("fixed_dt", [False, True])
def test_graph_capture_replays_match_eager(fixed_dt):
    """Two steps recorded into a HIP graph on the patch's own stream: each of
    three replays (with eager work and synchronisation between them) gives
    bitwise the state of the same two steps run eagerly."""
    say(f"graph capture, fixed dt {fixed_dt}")
    f = fields(24, seed=5, v_rms=1.0)
    s = torch.cuda.Stream()
    p = B.Patch(B.config(24), stream=s)
    p.init_from_potential(f.rho, f.v, f.A, f.P0, f.B0)
    st0 = p.state()
    dt = 0.9 * p.compute_dt() if fixed_dt else None
    for _ in range(2):
        p.step() if dt is None else p.step_dt(dt)
    ref = p.state()
    g = p.capture(2, dt)
    for r in range(3):
        p.set_state(st0["rho"], st0["m"], st0["E"], st0["b"])
        x = torch.randn(512, 512, device="cuda", dtype=torch.float64)
        x = x @ x
        torch.cuda.synchronize()
        g.replay()
        got = p.state()
        for k in ref:
            assert torch.equal(got[k], ref[k]), (r, k)
    with pytest.raises(ValueError):
        B.Patch(B.config(8)).capture(1)


@pytest.mark.parametrize("variant", ["planted", "nan_energy", "nan_density"])
def test_diagnostics_parity_hand_state(variant):
    """wm_diagnostics against the oracle on the hand-built 8^3 state of the
    oracle pins (gamma = 1.5): planted minimum density, a negative-pressure
    zone, a planted divergence of 2^-7, known totals; then with a NaN energy
    or a NaN density in one more zone."""
    say(f"diagnostics parity, hand state ({variant})")
    U, cfg = diag_state()
    if variant == "nan_energy":
        U["E"][1, 1, 1] = float("nan")
    elif variant == "nan_density":
        U["rho"][2, 3, 4] = float("nan")
    p = B.Patch(B.config(8, gamma=cfg.gamma))
    p.set_state(U["rho"], U["m"], U["E"], U["b"])
    g = p.diagnostics(raise_unphysical=False)
    o = mhd.diagnostics(U, cfg)
    assert_diag_parity(g, o, U, cfg.h)
    assert g["n_unphysical"] == {"planted": 1, "nan_energy": 2, "nan_density": 2}[variant]
    assert g["max_divb"] == 2.0 ** -7
