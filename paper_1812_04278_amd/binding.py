"""ctypes binding of libwenomhd.so (C ABI in include/wenomhd.h).

Argument marshalling only: every step of the method runs in the HIP library.
PyTorch provides the device memory and the stream.  Loading fails loudly when
the library has not been built; there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwenomhd.so")

WM_OK, WM_ERR_ARG, WM_ERR_HIP, WM_ERR_UNPHYSICAL, WM_ERR_STATE = 0, -1, -2, -3, -4
WM_FP64, WM_MIXED, WM_MIXED_F32STATE = 0, 1, 2
WM_WENO_JS, WM_WENO_Z, WM_WENO_Z_PRINTED = 0, 1, 2
WM_SSPRK3, WM_RK4 = 0, 1

SYMBOLS = [
    "wm_config_default", "wm_scratch_bytes", "wm_patch_create", "wm_patch_destroy", "wm_bind_state",
    "wm_init_from_potential", "wm_refresh_zone_field", "wm_compute_dt", "wm_rk_stage", "wm_step", "wm_diagnostics",
    "wm_debug_sweep", "wm_debug_wide_addressing", "wm_debug_rhs", "wm_adjoint_scratch_bytes", "wm_rhs_vjp", "wm_adjoint_step",
    "wm_step_record", "wm_zone_field_vjp", "wm_init_adjoint", "wm_profile", "wm_profile_report", "wm_last_error",
    "wm_step_static",
]
KERNEL_CLASSES = ["sweep", "update", "bcell", "dt", "other"]


class WmConfig(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("nz", ctypes.c_int),
                ("h", ctypes.c_double), ("gamma", ctypes.c_double), ("cfl", ctypes.c_double),
                ("eps_weno", ctypes.c_double), ("eps_B", ctypes.c_double), ("eps_Z", ctypes.c_double),
                ("weights", ctypes.c_int), ("precision", ctypes.c_int), ("integrator", ctypes.c_int),
                ("walls", ctypes.c_int * 3), ("rho_floor", ctypes.c_double), ("p_floor", ctypes.c_double)]


class WmDiag(ctypes.Structure):
    _fields_ = [("max_divb", ctypes.c_double), ("mass", ctypes.c_double), ("mom", ctypes.c_double * 3),
                ("energy", ctypes.c_double), ("bflux", ctypes.c_double * 3), ("min_rho", ctypes.c_double),
                ("min_p", ctypes.c_double), ("n_unphysical", ctypes.c_longlong), ("n_floored", ctypes.c_longlong)]

    def as_dict(self):
        return dict(max_divb=self.max_divb, mass=self.mass, mom=list(self.mom), energy=self.energy,
                    bflux=list(self.bflux), min_rho=self.min_rho, min_p=self.min_p,
                    n_unphysical=int(self.n_unphysical), n_floored=int(self.n_floored))


_lib = None


def load(path: str = LIB_PATH):
    """Loads the library (once) and declares the signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library {path} is missing: build it with `python -m paper_1812_04278_amd.build`")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    C = ctypes.POINTER(WmConfig)
    D = ctypes.POINTER(ctypes.c_double)
    lib.wm_config_default.argtypes = [C, ctypes.c_int]
    lib.wm_config_default.restype = None
    lib.wm_scratch_bytes.argtypes = [C]
    lib.wm_scratch_bytes.restype = ctypes.c_size_t
    lib.wm_patch_create.argtypes = [C, P, P, ctypes.c_size_t, ctypes.POINTER(P)]
    lib.wm_patch_destroy.argtypes = [P]
    lib.wm_bind_state.argtypes = [P, P, P, P]
    lib.wm_init_from_potential.argtypes = [P, P, P, P, ctypes.c_double, D]
    lib.wm_refresh_zone_field.argtypes = [P]
    lib.wm_compute_dt.argtypes = [P, D]
    lib.wm_rk_stage.argtypes = [P, ctypes.c_int, D]
    lib.wm_step.argtypes = [P, D]
    lib.wm_diagnostics.argtypes = [P, ctypes.POINTER(WmDiag)]
    lib.wm_debug_sweep.argtypes = [P, ctypes.c_int, P]
    lib.wm_debug_wide_addressing.argtypes = [P, ctypes.c_int]
    lib.wm_debug_rhs.argtypes = [P, P]
    lib.wm_adjoint_scratch_bytes.argtypes = [C]
    lib.wm_adjoint_scratch_bytes.restype = ctypes.c_size_t
    lib.wm_rhs_vjp.argtypes = [P, P, P, P, P, P]
    lib.wm_adjoint_step.argtypes = [P, P, P, P, P, P, ctypes.c_double, P, P]
    lib.wm_step_record.argtypes = [P, ctypes.c_double, P, P]
    lib.wm_zone_field_vjp.argtypes = [P, P, P]
    lib.wm_init_adjoint.argtypes = [P, P, P, P, P, D, P, P, P, P]
    lib.wm_profile.argtypes = [P, ctypes.c_int]
    lib.wm_profile_report.argtypes = [P, D, ctypes.c_int]
    lib.wm_step_static.argtypes = [C, P, P, P, P, D]
    lib.wm_last_error.argtypes = []
    lib.wm_last_error.restype = ctypes.c_char_p
    for name in ("wm_patch_create", "wm_patch_destroy", "wm_bind_state", "wm_init_from_potential",
                 "wm_refresh_zone_field",
                 "wm_compute_dt", "wm_rk_stage", "wm_step", "wm_diagnostics", "wm_debug_sweep",
                 "wm_debug_wide_addressing", "wm_debug_rhs",
                 "wm_rhs_vjp", "wm_adjoint_step", "wm_step_record", "wm_zone_field_vjp", "wm_init_adjoint",
                 "wm_profile", "wm_profile_report", "wm_step_static"):
        getattr(lib, name).restype = ctypes.c_int
    _lib = lib
    return lib


class WmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"wenomhd status {status}: {msg}")
        self.status = status


def _check(status):
    if status != WM_OK:
        raise WmError(status, load().wm_last_error().decode())


def config(n=None, nx=None, ny=None, nz=None, h=None, gamma=5.0 / 3.0, cfl=0.4, eps=1e-6, eps_B=1e-30,
           eps_Z=1e-40, weights=WM_WENO_JS, precision=WM_FP64, integrator=WM_SSPRK3, walls=(0, 0, 0),
           rho_floor=0.0, p_floor=0.0) -> WmConfig:
    nx = nx or n
    ny = ny or n
    nz = nz or n
    c = WmConfig(nx=nx, ny=ny, nz=nz, h=h if h is not None else 1.0 / nx, gamma=gamma, cfl=cfl,
                 eps_weno=eps, eps_B=eps_B, eps_Z=eps_Z, weights=weights, precision=precision,
                 integrator=integrator, walls=(ctypes.c_int * 3)(*[int(w) for w in walls]),
                 rho_floor=rho_floor, p_floor=p_floor)
    return c


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


def step_static(cfg: WmConfig, hydro: torch.Tensor, bface: torch.Tensor, bcell: torch.Tensor,
                stream: torch.cuda.Stream | None = None, want_dt: bool = False):
    """wm_step_static: one step of the given state tensors in place, with the
    library's static device scratch (no allocation by the library or here).
    Returns the step's dt when ``want_dt`` (synchronises the stream)."""
    lib = load()
    for t in (hydro, bface, bcell):
        if not t.is_contiguous():
            raise ValueError("state tensors must be contiguous")
    s = stream or torch.cuda.current_stream(hydro.device)
    d = ctypes.c_double() if want_dt else None
    _check(lib.wm_step_static(ctypes.byref(cfg), ctypes.c_void_p(s.cuda_stream), _ptr(hydro), _ptr(bface),
                              _ptr(bcell), ctypes.byref(d) if want_dt else None))
    return d.value if want_dt else None


def _on_stream(fn):
    """Runs a Patch method with the patch's stream current, so the torch copies
    and allocations it makes are ordered with the library's launches."""
    def wrapped(self, *a, **kw):
        with torch.cuda.stream(self.stream):
            return fn(self, *a, **kw)
    wrapped.__name__, wrapped.__doc__ = fn.__name__, fn.__doc__
    return wrapped


class _StepGraph:
    """Captured steps of a patch; ``replay()`` launches them on the patch's
    stream (torch replays a graph on the current stream)."""

    def __init__(self, graph, stream):
        self.graph, self.stream = graph, stream

    def replay(self):
        with torch.cuda.stream(self.stream):
            self.graph.replay()


class Patch:
    """A periodic box on one GPU: state tensors, scratch and the C patch handle.

    State (on ``device``; float64, or float32 for WM_MIXED_F32STATE): ``hydro``
    [5, nz, ny, nx] (rho, m, E), ``bface`` [3, nz, ny, nx], ``bcell`` [3, nz, ny, nx].

    Every launch of the patch goes to ``stream`` (default: the current stream
    when the patch is created), and the methods below make their own torch
    copies on it too.  Device tensors passed in must be ready on that stream;
    tensors returned, and the state, are ready on it."""

    def __init__(self, cfg: WmConfig, device="cuda", stream: torch.cuda.Stream | None = None):
        self.lib = load()
        self.cfg = cfg
        self.device = torch.device(device)
        shape = (cfg.nz, cfg.ny, cfg.nx)
        self.shape = shape
        nbytes = self.lib.wm_scratch_bytes(ctypes.byref(cfg))
        if nbytes == 0:
            raise WmError(WM_ERR_ARG, "invalid configuration")
        self.scratch = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.dtype = torch.float32 if cfg.precision == WM_MIXED_F32STATE else torch.float64
        self.hydro = torch.zeros((5,) + shape, dtype=self.dtype, device=self.device)
        self.bface = torch.zeros((3,) + shape, dtype=self.dtype, device=self.device)
        self.bcell = torch.zeros((3,) + shape, dtype=self.dtype, device=self.device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        h = ctypes.c_void_p()
        _check(self.lib.wm_patch_create(ctypes.byref(cfg), ctypes.c_void_p(self.stream.cuda_stream),
                                        _ptr(self.scratch), nbytes, ctypes.byref(h)))
        self.handle = h
        _check(self.lib.wm_bind_state(h, _ptr(self.hydro), _ptr(self.bface), _ptr(self.bcell)))

    def close(self):
        if getattr(self, "handle", None):
            self.lib.wm_patch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- state
    @_on_stream
    def init_from_potential(self, rho, v, A, P0: float, B0):
        dev = lambda x: torch.as_tensor(x, dtype=torch.float64).to(self.device).contiguous()
        r, vv, AA = dev(rho), dev(v), dev(A)
        assert r.shape == self.shape and vv.shape == (3,) + self.shape and AA.shape == (3,) + self.shape
        b0 = (ctypes.c_double * 3)(*[float(x) for x in B0])
        _check(self.lib.wm_init_from_potential(self.handle, _ptr(r), _ptr(vv), _ptr(AA), float(P0), b0))
        self.stream.synchronize()   # the inputs r, vv, AA are freed on return

    @_on_stream
    def set_state(self, rho, m, E, b):
        """Loads a conserved state (rho, m, E, face b) and re-derives zone B."""
        with torch.no_grad():
            self.hydro[0].copy_(torch.as_tensor(rho))
            self.hydro[1:4].copy_(torch.as_tensor(m))
            self.hydro[4].copy_(torch.as_tensor(E))
            self.bface.copy_(torch.as_tensor(b))
        _check(self.lib.wm_refresh_zone_field(self.handle))

    @_on_stream
    def state(self):
        """Host copy (float64) as the oracle's dict (rho, m, E, b)."""
        h = self.hydro.cpu().double()
        return dict(rho=h[0], m=h[1:4].clone(), E=h[4], b=self.bface.cpu().double())

    # ---- method
    def compute_dt(self) -> float:
        d = ctypes.c_double()
        _check(self.lib.wm_compute_dt(self.handle, ctypes.byref(d)))
        return d.value

    def rk_stage(self, stage: int, dt: float | None = None):
        if dt is None:
            _check(self.lib.wm_rk_stage(self.handle, stage, None))
        else:
            d = ctypes.c_double(dt)
            _check(self.lib.wm_rk_stage(self.handle, stage, ctypes.byref(d)))

    def step(self, want_dt: bool = False):
        if want_dt:
            d = ctypes.c_double()
            _check(self.lib.wm_step(self.handle, ctypes.byref(d)))
            return d.value
        _check(self.lib.wm_step(self.handle, None))
        return None

    def capture(self, nsteps: int = 1, dt: float | None = None):
        """Records ``nsteps`` steps into a HIP graph (a ``torch.cuda.CUDAGraph``)
        and returns a handle whose ``replay()`` runs them with one launch on the
        patch's stream, ordered like every other call of the patch.  dt: None
        for eq. (cfl) on the device at every step, or a fixed value.  The patch
        must own a stream other than the default one.  A step launches only
        kernels (no copies, memsets or host synchronisation), so the graph
        replays exactly what the eager calls would run."""
        if self.stream == torch.cuda.default_stream(self.device):
            raise ValueError("graph capture needs a patch created with its own stream")
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=self.stream):
            for _ in range(nsteps):
                if dt is None:
                    _check(self.lib.wm_step(self.handle, None))
                else:
                    self.step_dt(dt)
        return _StepGraph(g, self.stream)

    @property
    def n_stages(self) -> int:
        return 4 if self.cfg.integrator == WM_RK4 else 3

    def step_dt(self, dt: float):
        for s in range(self.n_stages):
            self.rk_stage(s, dt)

    def diagnostics(self, raise_unphysical: bool = True):
        d = WmDiag()
        st = self.lib.wm_diagnostics(self.handle, ctypes.byref(d))
        if st != WM_OK and (raise_unphysical or st != WM_ERR_UNPHYSICAL):
            _check(st)
        return d.as_dict()

    def debug_wide_addressing(self, on: bool = True) -> None:
        """Testing switch: the sweep uses 64-bit addresses (its path for arrays of 4 GiB or more)."""
        _check(self.lib.wm_debug_wide_addressing(self.handle, int(bool(on))))

    @_on_stream
    def debug_sweep(self, axis: int) -> torch.Tensor:
        out = torch.empty((9,) + self.shape, dtype=torch.float64, device=self.device)
        _check(self.lib.wm_debug_sweep(self.handle, axis, _ptr(out)))
        return out

    @_on_stream
    def debug_rhs(self) -> torch.Tensor:
        out = torch.empty((8,) + self.shape, dtype=torch.float64, device=self.device)
        _check(self.lib.wm_debug_rhs(self.handle, _ptr(out)))
        return out

    def profile(self, enable: bool):
        _check(self.lib.wm_profile(self.handle, 1 if enable else 0))

    def profile_report(self):
        """{kernel class: (launches, total ms)} of the current timing session."""
        out = (ctypes.c_double * 10)()
        _check(self.lib.wm_profile_report(self.handle, out, 10))
        return {name: (int(out[2 * c]), float(out[2 * c + 1])) for c, name in enumerate(KERNEL_CLASSES)}

    # ---- adjoint
    def _adj(self):
        if getattr(self, "adj_scratch", None) is None:
            nbytes = self.lib.wm_adjoint_scratch_bytes(ctypes.byref(self.cfg))
            self.adj_scratch = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        return self.adj_scratch

    @_on_stream
    def rhs_vjp(self, hydro, bface, lam_k):
        """(dL/dU)^T lam_k at U = (hydro, bface); lam_k [8, nz, ny, nx]."""
        out = torch.empty((8,) + self.shape, dtype=torch.float64, device=self.device)
        h, b, l = hydro.contiguous(), bface.contiguous(), lam_k.contiguous()
        _check(self.lib.wm_rhs_vjp(self.handle, _ptr(self._adj()), _ptr(h), _ptr(b), _ptr(l), _ptr(out)))
        return out

    @_on_stream
    def adjoint_step(self, Un_hydro, Un_bface, dt: float, lam_hydro, lam_bface, U1=None, U2=None):
        """In place: (lam_hydro, lam_bface) <- adjoint of one step from U^n with dt.
        U1, U2: the step's stage states from step_record ([8, nz, ny, nx]), or
        None to recompute them."""
        if (U1 is None) != (U2 is None):
            raise ValueError("give both stage states or neither")
        _check(self.lib.wm_adjoint_step(self.handle, _ptr(self._adj()), _ptr(Un_hydro), _ptr(Un_bface),
                                        _ptr(U1) if U1 is not None else None,
                                        _ptr(U2) if U2 is not None else None,
                                        float(dt), _ptr(lam_hydro), _ptr(lam_bface)))

    @_on_stream
    def step_record(self, dt: float, U1=None, U2=None):
        """One step of the bound state with dt; returns its two stage states
        ([8, nz, ny, nx] each, written into U1/U2 when given)."""
        if U1 is None:
            U1 = torch.empty((8,) + self.shape, dtype=self.dtype, device=self.device)
        if U2 is None:
            U2 = torch.empty((8,) + self.shape, dtype=self.dtype, device=self.device)
        if U1.dtype != self.dtype or U2.dtype != self.dtype:
            raise ValueError("stage states must have the state's dtype")
        _check(self.lib.wm_step_record(self.handle, float(dt), _ptr(U1), _ptr(U2)))
        return U1, U2

    @_on_stream
    def zone_field_vjp(self, lam_bcell, lam_bface):
        _check(self.lib.wm_zone_field_vjp(self.handle, _ptr(lam_bcell.contiguous()), _ptr(lam_bface)))

    @_on_stream
    def init_adjoint(self, rho, v, A, B0, lam_hydro, lam_bface):
        """Gradients (g_A, g_v) of the initial-state map for cotangents of the state."""
        dev = lambda x: torch.as_tensor(x, dtype=torch.float64).to(self.device).contiguous()
        r, vv, AA = dev(rho), dev(v), dev(A)
        gA = torch.empty((3,) + self.shape, dtype=torch.float64, device=self.device)
        gv = torch.empty((3,) + self.shape, dtype=torch.float64, device=self.device)
        b0 = (ctypes.c_double * 3)(*[float(x) for x in B0])
        _check(self.lib.wm_init_adjoint(self.handle, _ptr(self._adj()), _ptr(r), _ptr(vv), _ptr(AA), b0,
                                        _ptr(lam_hydro.contiguous()), _ptr(lam_bface.contiguous()), _ptr(gA),
                                        _ptr(gv)))
        self.stream.synchronize()
        return gA, gv

