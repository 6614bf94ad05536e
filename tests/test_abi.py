"""Host-only checks of the C ABI: the library loads, exports every function the
header declares, and validates arguments before touching a GPU."""
import ctypes
import os
import re

import pytest

from paper_1812_04278_amd import binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "wenomhd.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(wm_[a-z_0-9]+)\s*\(", text)))


def test_header_lists_the_binding_symbols():
    assert declared_functions() == sorted(B.SYMBOLS)


def test_library_exports_every_declared_symbol():
    lib = B.load()
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_clock_build_exports_its_call():
    """The phase-clock measurement build exports the call of its own header;
    the product library does not."""
    from paper_1812_04278_amd import build
    text = open(os.path.join(ROOT, "include", "wenomhd_clock.h")).read()
    names = sorted(set(re.findall(r"\b(wm_[a-z_0-9]+)\s*\(", re.sub(r"/\*.*?\*/", "", text, flags=re.S))))
    assert names == ["wm_clock_sweep_buffer"]
    if not os.path.exists(build.CLOCK_LIB):
        pytest.skip("clock build not present")
    clk = ctypes.CDLL(build.CLOCK_LIB)
    assert hasattr(clk, "wm_clock_sweep_buffer")
    clk.wm_clock_sweep_buffer.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_size_t]
    assert clk.wm_clock_sweep_buffer(3, None, 0) != 0          # invalid axis, no GPU touched
    assert clk.wm_clock_sweep_buffer(0, None, 0) == 0          # unregister
    assert not hasattr(B.load(), "wm_clock_sweep_buffer")


def test_scratch_bytes_and_default_config():
    lib = B.load()
    c = B.WmConfig()
    lib.wm_config_default(ctypes.byref(c), 32)
    assert (c.nx, c.ny, c.nz) == (32, 32, 32)
    assert abs(c.h - 1 / 32) < 1e-18 and abs(c.gamma - 5 / 3) < 1e-15 and c.cfl == 0.4
    assert c.eps_weno == 1e-6 and c.eps_B == 1e-30
    assert c.integrator == B.WM_SSPRK3
    n = lib.wm_scratch_bytes(ctypes.byref(c))
    N = 32 ** 3
    assert n >= 40 * N * 8 and n % 256 == 0
    c2 = B.config(nx=20, ny=9, nz=5)
    assert lib.wm_scratch_bytes(ctypes.byref(c2)) >= 40 * 20 * 9 * 5 * 8


@pytest.mark.parametrize("field,value", [("nx", 0), ("h", 0.0), ("gamma", 1.0), ("cfl", -1.0),
                                         ("weights", 3), ("weights", -1), ("precision", 9), ("eps_weno", 0.0),
                                         ("integrator", 2), ("eps_Z", 1e-60)])
def test_invalid_config_rejected(field, value):
    lib = B.load()
    c = B.config(16)
    setattr(c, field, value)
    assert lib.wm_scratch_bytes(ctypes.byref(c)) == 0
    h = ctypes.c_void_p()
    st = lib.wm_patch_create(ctypes.byref(c), None, ctypes.c_void_p(256), 1 << 40, ctypes.byref(h))
    assert st == B.WM_ERR_ARG
    assert lib.wm_last_error().decode().startswith("invalid config")


@pytest.mark.parametrize("kw", [dict(walls=(1, 0, 0), nx=2), dict(walls=(0, 2, 0)), dict(rho_floor=-1.0),
                                dict(p_floor=float("nan")), dict(rho_floor=0.1, integrator=1)])
def test_invalid_walls_and_floors_rejected(kw):
    """A walled axis needs three zones (the mirror stencil), walls are 0 or 1,
    floors are finite and non-negative and apply to the SSP-RK3 stages."""
    lib = B.load()
    args = dict(n=16)
    args.update(kw)
    c = B.config(**args)
    assert lib.wm_scratch_bytes(ctypes.byref(c)) == 0


def test_walls_and_floors_accepted():
    lib = B.load()
    c = B.config(16, walls=(1, 0, 1), rho_floor=1e-3, p_floor=1e-4)
    assert lib.wm_scratch_bytes(ctypes.byref(c)) > lib.wm_scratch_bytes(ctypes.byref(B.config(16))) - 1


def test_patch_create_argument_errors():
    lib = B.load()
    c = B.config(16)
    need = lib.wm_scratch_bytes(ctypes.byref(c))
    h = ctypes.c_void_p()
    assert lib.wm_patch_create(ctypes.byref(c), None, None, need, ctypes.byref(h)) == B.WM_ERR_ARG
    assert lib.wm_patch_create(ctypes.byref(c), None, ctypes.c_void_p(4096 + 8), need, ctypes.byref(h)) == B.WM_ERR_ARG
    assert lib.wm_patch_create(ctypes.byref(c), None, ctypes.c_void_p(4096), need - 1, ctypes.byref(h)) == B.WM_ERR_ARG
    # a fake aligned address is accepted at creation (nothing is launched); then calls
    # before binding the state fail with WM_ERR_STATE without launching anything
    assert lib.wm_patch_create(ctypes.byref(c), None, ctypes.c_void_p(4096), need, ctypes.byref(h)) == B.WM_OK
    d = ctypes.c_double()
    assert lib.wm_compute_dt(h, ctypes.byref(d)) == B.WM_ERR_STATE
    assert lib.wm_step(h, None) == B.WM_ERR_STATE
    assert lib.wm_rk_stage(h, 0, None) == B.WM_ERR_STATE
    assert lib.wm_bind_state(h, None, None, None) == B.WM_ERR_ARG
    # bind fake addresses: order and argument checks still happen on the host
    fake = ctypes.c_void_p(1 << 20)
    assert lib.wm_bind_state(h, fake, fake, fake) == B.WM_OK
    assert lib.wm_rk_stage(h, 3, None) == B.WM_ERR_ARG
    assert lib.wm_rk_stage(h, 1, None) == B.WM_ERR_STATE          # stage 1 before stage 0
    assert lib.wm_rk_stage(h, 0, None) == B.WM_ERR_STATE          # no dt yet
    nan = ctypes.c_double(float("nan"))
    assert lib.wm_rk_stage(h, 0, ctypes.byref(nan)) == B.WM_ERR_ARG
    assert lib.wm_debug_sweep(h, 5, fake) == B.WM_ERR_ARG
    assert lib.wm_patch_destroy(h) == B.WM_OK


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(RuntimeError, match="missing"):
        B._lib_saved = B._lib
        try:
            B._lib = None
            B.load(str(tmp_path / "nope.so"))
        finally:
            B._lib = B._lib_saved


@pytest.mark.parametrize("w", [0, 1, 2])
def test_all_weights_accepted(w):
    """Jiang-Shu, WENO-Z of reading R13 and WENO-Z as printed are valid configurations."""
    lib = B.load()
    c = B.config(16, weights=w)
    assert w == (B.WM_WENO_JS, B.WM_WENO_Z, B.WM_WENO_Z_PRINTED)[w]
    assert lib.wm_scratch_bytes(ctypes.byref(c)) > 0
