"""Thin Python binding of libfvrk3.so (include/fvrk3.h).

Argument marshalling only: every step of the path runs in the HIP library.
PyTorch supplies device memory (tensors) and the current HIP stream.  The
library must be built (``python -m paper_2402_05193_amd.build``); importing
this module without it raises immediately -- there is no fallback.
"""
from __future__ import annotations

import contextlib
import ctypes
import os
from dataclasses import dataclass, field

import torch

EULER, NS, DIM = 0, 1, 2
F64, F32 = 0, 1
PERIODIC, ZERO_GRADIENT, SYMMETRY = 0, 1, 2
CASE_UNIFORM, CASE_TGV, CASE_RIEMANN, CASE_SBI, CASE_GAUSS_WAVE, CASE_ISENTROPIC_VORTEX = 0, 1, 2, 3, 4, 5
ABI_VERSION = 3

OK, EINVAL, ENULL, EALIGN, EUNSUPPORTED, EHIP, EINADMISSIBLE, ENONFINITE = 0, -1, -2, -3, -4, -5, -6, -7

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("FVRK3_LIB", os.path.join(_HERE, "libfvrk3.so"))

EXPORTED = ["fv_ncomp", "workspace_bytes", "init_state", "prim_to_cons", "cons_to_prim", "rhs", "rhs_ws",
            "limiter_flag_bytes", "rhs_flags", "rk3_stage",
            "rk3_stage3_cfl", "rk3_step", "compute_dt", "advance", "advance_noalloc", "rhs_adjoint", "adjoint_workspace_bytes",
            "rk3_step_adjoint", "rk3_step_adjoint_stages", "check_state", "workspace_time",
            "batch_table_bytes", "batch_create", "batch_destroy", "batch_set", "batch_step", "batch_step_graph",
            "batch_graph_count", "stage_workgroups", "last_error"]


class FVError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_int32),
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("model", ctypes.c_int32), ("dtype", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 6),
        ("positivity", ctypes.c_int32), ("recon", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("gamma1", ctypes.c_double), ("pinf1", ctypes.c_double),
        ("gamma2", ctypes.c_double), ("pinf2", ctypes.c_double),
        ("mu", ctypes.c_double), ("prandtl", ctypes.c_double),
        ("eps_rho", ctypes.c_double), ("eps_rhoc2", ctypes.c_double), ("eps_alpha", ctypes.c_double),
        ("weno_eps", ctypes.c_double),
        ("cfl", ctypes.c_double),
        ("visc_law", ctypes.c_int32), ("scheme", ctypes.c_int32),
        ("T_ref", ctypes.c_double), ("sutherland", ctypes.c_double), ("gas_R", ctypes.c_double),
        ("visc_order", ctypes.c_int32), ("thinc", ctypes.c_int32),
    ]


class Report(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("bad_count_clamped", ctypes.c_int32),
                ("first_bad_cell", ctypes.c_int64)]


@dataclass
class Config:
    """Problem description mirrored into ``fv_config``."""
    nx: int
    ny: int
    nz: int
    dx: float = 1.0
    dy: float = 1.0
    dz: float = 1.0
    model: int = EULER
    dtype: int = F64
    bc: tuple = (PERIODIC,) * 6
    gamma1: float = 1.4
    pinf1: float = 0.0
    gamma2: float = 1.4
    pinf2: float = 0.0
    mu: float = 0.0
    prandtl: float = 0.72
    positivity: int = -1
    eps_rho: float = 0.0
    eps_rhoc2: float = 0.0
    eps_alpha: float = 0.0
    weno_eps: float = 0.0
    cfl: float = 0.5
    recon: int = 0          # 0: primitive variables, 1: characteristic variables
    scheme: int = 0         # 0: WENO5-Z, 1: TENO6-A
    visc_order: int = 0     # central viscous stencils: 0/4 fused 4th order, 6 sixth order (separate passes)
    thinc: int = 0          # five-equation model: THINC interface capturing
    visc_law: int = 0       # 0: constant mu, 1: power law, 2: Sutherland (Sec. 2.5)
    T_ref: float = 1.0
    sutherland: float = 0.0
    gas_R: float = 1.0

    @property
    def ncomp(self) -> int:
        return 7 if self.model == DIM else 5

    @property
    def shape(self):
        return (self.ncomp, self.nz, self.ny, self.nx)

    @property
    def torch_dtype(self):
        return torch.float64 if self.dtype == F64 else torch.float32

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    def c_struct(self) -> _Cfg:
        c = _Cfg()
        c.abi_version = ABI_VERSION
        c.nx, c.ny, c.nz = self.nx, self.ny, self.nz
        c.model, c.dtype = self.model, self.dtype
        for i, b in enumerate(self.bc):
            c.bc[i] = int(b)
        c.positivity, c.recon = self.positivity, self.recon
        c.dx, c.dy, c.dz = self.dx, self.dy, self.dz
        c.gamma1, c.pinf1, c.gamma2, c.pinf2 = self.gamma1, self.pinf1, self.gamma2, self.pinf2
        c.mu, c.prandtl = self.mu, self.prandtl
        c.eps_rho, c.eps_rhoc2, c.eps_alpha = self.eps_rho, self.eps_rhoc2, self.eps_alpha
        c.weno_eps, c.cfl = self.weno_eps, self.cfl
        c.visc_law, c.scheme = self.visc_law, self.scheme
        c.T_ref, c.sutherland, c.gas_R = self.T_ref, self.sutherland, self.gas_R
        c.visc_order, c.thinc = self.visc_order, self.thinc
        return c


_lib = None


def load(path: str):
    """Open a build of the library at ``path`` and declare its entry points (raises if
    it has not been built)."""
    if not os.path.exists(path):
        raise ImportError(f"{path} is missing: build it with `python -m paper_2402_05193_amd.build`")
    return _declare(ctypes.CDLL(path))


def lib():
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        _lib = load(LIB_PATH)
    return _lib


@contextlib.contextmanager
def using(L):
    """Within the block every call of this module goes to the library ``L`` (from
    ``load``), e.g. a build with another tile shape."""
    global _lib
    saved = lib()
    _lib = L
    try:
        yield L
    finally:
        _lib = saved


def _declare(L):
    """Declare the argument and result types of every entry point of L."""
    cp = ctypes.POINTER(_Cfg)
    vp = ctypes.c_void_p
    L.fv_ncomp.argtypes = [cp]
    L.workspace_bytes.argtypes = [cp, ctypes.POINTER(ctypes.c_size_t)]
    L.init_state.argtypes = [cp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                             ctypes.c_uint64, vp, vp]
    L.prim_to_cons.argtypes = [cp, vp, vp, vp]
    L.cons_to_prim.argtypes = [cp, vp, vp, vp]
    L.rhs.argtypes = [cp, vp, vp, ctypes.c_double, vp]
    L.rhs_ws.argtypes = [cp, vp, vp, ctypes.c_double, vp, vp]
    L.limiter_flag_bytes.argtypes = [cp, ctypes.POINTER(ctypes.c_size_t)]
    L.rhs_flags.argtypes = [cp, vp, vp, ctypes.c_double, vp, vp, vp]
    L.rk3_stage.argtypes = [cp, ctypes.c_int32, vp, vp, vp, ctypes.c_double, vp, vp]
    L.rk3_stage3_cfl.argtypes = [cp, vp, vp, vp, vp, vp, vp, vp]
    L.rk3_step.argtypes = [cp, vp, ctypes.c_double, vp, vp]
    L.compute_dt.argtypes = [cp, vp, vp, vp, vp]
    L.advance.argtypes = [cp, vp, ctypes.c_int32, ctypes.c_double, ctypes.POINTER(ctypes.c_double), vp, vp]
    L.advance_noalloc.argtypes = [cp, vp, ctypes.c_int32, ctypes.c_double, vp]
    L.rhs_adjoint.argtypes = [cp, vp, vp, vp, vp, vp]
    L.adjoint_workspace_bytes.argtypes = [cp, ctypes.POINTER(ctypes.c_size_t)]
    L.rk3_step_adjoint.argtypes = [cp, vp, vp, ctypes.c_double, vp, vp]
    L.rk3_step_adjoint_stages.argtypes = [cp, vp, vp, vp, vp, ctypes.c_double, vp, vp]
    L.check_state.argtypes = [cp, vp, vp, ctypes.POINTER(Report), vp]
    L.workspace_time.argtypes = [cp, vp, ctypes.POINTER(ctypes.c_double), vp]
    L.batch_table_bytes.argtypes = [ctypes.c_int32, ctypes.POINTER(ctypes.c_size_t)]
    L.batch_create.argtypes = [ctypes.c_int32, vp, ctypes.c_size_t, ctypes.POINTER(vp)]
    L.batch_destroy.argtypes = [vp]
    L.batch_set.argtypes = [vp, ctypes.c_int32, cp, ctypes.POINTER(vp), ctypes.POINTER(vp),
                            ctypes.POINTER(ctypes.c_int32), vp]
    L.batch_step.argtypes = [vp, ctypes.c_int32, vp]
    L.batch_step_graph.argtypes = [vp, ctypes.c_int32, vp]
    L.batch_graph_count.argtypes = [vp]
    L.stage_workgroups.argtypes = [cp, ctypes.POINTER(ctypes.c_int32)]
    L.last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("last_error",):
            getattr(L, name).restype = ctypes.c_int
    return L


def _check(code: int):
    if code != OK:
        raise FVError(code, lib().last_error().decode())
    return code


def _ptr(t) -> int | None:
    if t is None:
        return None
    if isinstance(t, int):
        return t
    return t.data_ptr()


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _state(cfg: Config, t: torch.Tensor, name: str):
    if t.dtype != cfg.torch_dtype or not t.is_contiguous() or t.numel() != cfg.ncomp * cfg.ncells:
        raise ValueError(f"{name}: expected a contiguous {cfg.torch_dtype} tensor of {cfg.shape}")
    if not t.is_cuda:
        raise ValueError(f"{name}: must be a device tensor")


# ------------------------------------------------------------------ API
def ncomp(cfg: Config) -> int:
    c = cfg.c_struct()
    r = lib().fv_ncomp(ctypes.byref(c))
    if r < 0:
        _check(r)
    return r


def workspace_bytes(cfg: Config) -> int:
    c = cfg.c_struct()
    out = ctypes.c_size_t(0)
    _check(lib().workspace_bytes(ctypes.byref(c), ctypes.byref(out)))
    return out.value


def empty_state(cfg: Config, device="cuda") -> torch.Tensor:
    return torch.empty(cfg.shape, dtype=cfg.torch_dtype, device=device)


def workspace(cfg: Config, device="cuda") -> torch.Tensor:
    return torch.empty(workspace_bytes(cfg), dtype=torch.uint8, device=device)


def init_state(cfg: Config, case_id: int, params, U: torch.Tensor, seed: int = 0, stream=None):
    _state(cfg, U, "U")
    arr = (ctypes.c_double * max(1, len(params)))(*[float(p) for p in params])
    c = cfg.c_struct()
    _check(lib().init_state(ctypes.byref(c), int(case_id), arr, len(params), ctypes.c_uint64(seed & (2**64 - 1)),
                            _ptr(U), _stream(stream)))
    return U


def prim_to_cons(cfg: Config, W: torch.Tensor, U: torch.Tensor, stream=None):
    _state(cfg, W, "W")
    _state(cfg, U, "U")
    c = cfg.c_struct()
    _check(lib().prim_to_cons(ctypes.byref(c), _ptr(W), _ptr(U), _stream(stream)))
    return U


def cons_to_prim(cfg: Config, U: torch.Tensor, W: torch.Tensor, stream=None):
    _state(cfg, U, "U")
    _state(cfg, W, "W")
    c = cfg.c_struct()
    _check(lib().cons_to_prim(ctypes.byref(c), _ptr(U), _ptr(W), _stream(stream)))
    return W


def rhs(cfg: Config, U: torch.Tensor, R: torch.Tensor, dt: float = 0.0, stream=None, ws=None):
    """R = R_NSE(U); with a workspace (required for sixth-order viscous fluxes,
    allocated here if not given) through rhs_ws."""
    _state(cfg, U, "U")
    _state(cfg, R, "R")
    c = cfg.c_struct()
    if ws is None and cfg.visc_order == 6:
        ws = workspace(cfg)
    if ws is None:
        _check(lib().rhs(ctypes.byref(c), _ptr(U), _ptr(R), float(dt), _stream(stream)))
    else:
        _check(lib().rhs_ws(ctypes.byref(c), _ptr(U), _ptr(R), float(dt), _ptr(ws), _stream(stream)))
    return R


def limiter_flag_bytes(cfg: Config) -> int:
    c = cfg.c_struct()
    out = ctypes.c_size_t(0)
    _check(lib().limiter_flag_bytes(ctypes.byref(c), ctypes.byref(out)))
    return out.value


def rhs_flags(cfg: Config, U: torch.Tensor, R: torch.Tensor, dt: float = 0.0, flags: torch.Tensor | None = None,
              ws=None, stream=None):
    """R = R_NSE(U) and the limiter decisions of every face (uint8 tensor of
    limiter_flag_bytes(cfg) bytes: x faces [nz][ny][nx+1], then y [nz][ny+1][nx], then
    z [nz+1][ny][nx]; bit 0/1: interpolation limiter on the left/right state, bit 2:
    flux limiter).  Returns (R, [flags_x, flags_y, flags_z]) as views."""
    _state(cfg, U, "U")
    _state(cfg, R, "R")
    nb = limiter_flag_bytes(cfg)
    if flags is None:
        flags = torch.empty(nb, dtype=torch.uint8, device=U.device)
    if flags.dtype != torch.uint8 or not flags.is_contiguous() or flags.numel() != nb or not flags.is_cuda:
        raise ValueError(f"flags: expected a contiguous device uint8 tensor of {nb} bytes")
    if ws is None and cfg.visc_order == 6:
        ws = workspace(cfg)
    c = cfg.c_struct()
    _check(lib().rhs_flags(ctypes.byref(c), _ptr(U), _ptr(R), float(dt), _ptr(flags), _ptr(ws), _stream(stream)))
    nx, ny, nz = cfg.nx, cfg.ny, cfg.nz
    n0 = (nx + 1) * ny * nz
    n1 = nx * (ny + 1) * nz
    views = [flags[:n0].view(nz, ny, nx + 1), flags[n0:n0 + n1].view(nz, ny + 1, nx),
             flags[n0 + n1:].view(nz + 1, ny, nx)]
    return R, views


def rk3_stage(cfg: Config, stage: int, Un, Uk, Uout, dt: float = 0.0, dt_dev: torch.Tensor | None = None,
              stream=None):
    for t, n in ((Un, "Un"), (Uk, "Uk"), (Uout, "Uout")):
        _state(cfg, t, n)
    c = cfg.c_struct()
    _check(lib().rk3_stage(ctypes.byref(c), int(stage), _ptr(Un), _ptr(Uk), _ptr(Uout), float(dt), _ptr(dt_dev),
                           _stream(stream)))
    return Uout


def rk3_stage3_cfl(cfg: Config, Un, Uk, Uout, dt_dev: torch.Tensor, dt_next: torch.Tensor, ws: torch.Tensor,
                   stream=None):
    """Third stage fused with the CFL reduction of its output (writes dt_next on the device)."""
    for t, n in ((Un, "Un"), (Uk, "Uk"), (Uout, "Uout")):
        _state(cfg, t, n)
    c = cfg.c_struct()
    _check(lib().rk3_stage3_cfl(ctypes.byref(c), _ptr(Un), _ptr(Uk), _ptr(Uout), _ptr(dt_dev), _ptr(dt_next),
                                _ptr(ws), _stream(stream)))
    return Uout


def rk3_step(cfg: Config, U: torch.Tensor, dt: float, ws: torch.Tensor, stream=None):
    _state(cfg, U, "U")
    c = cfg.c_struct()
    _check(lib().rk3_step(ctypes.byref(c), _ptr(U), float(dt), _ptr(ws), _stream(stream)))
    return U


def compute_dt(cfg: Config, U: torch.Tensor, dt_dev: torch.Tensor, ws: torch.Tensor, stream=None):
    _state(cfg, U, "U")
    c = cfg.c_struct()
    _check(lib().compute_dt(ctypes.byref(c), _ptr(U), _ptr(dt_dev), _ptr(ws), _stream(stream)))
    return dt_dev


def advance(cfg: Config, U: torch.Tensor, nsteps: int, dt: float, ws: torch.Tensor, t: float | None = None,
            stream=None):
    """Advance in place; returns the new time if ``t`` is given (one host sync), else None."""
    _state(cfg, U, "U")
    c = cfg.c_struct()
    tp = None
    tv = None
    if t is not None:
        tv = ctypes.c_double(t)
        tp = ctypes.byref(tv)
    _check(lib().advance(ctypes.byref(c), _ptr(U), int(nsteps), float(dt), tp, _ptr(ws), _stream(stream)))
    return tv.value if tv is not None else None


NOALLOC_SCRATCH_BYTES = 64 << 20   # FV_NOALLOC_SCRATCH_BYTES of include/fvrk3.h


def advance_noalloc(cfg: Config, U: torch.Tensor, nsteps: int, dt: float, stream=None):
    """advance without a caller workspace and without any device allocation (the
    library's fixed per-device scratch array; problems whose workspace exceeds
    NOALLOC_SCRATCH_BYTES are rejected)."""
    _state(cfg, U, "U")
    c = cfg.c_struct()
    _check(lib().advance_noalloc(ctypes.byref(c), _ptr(U), int(nsteps), float(dt), _stream(stream)))
    return U


def rhs_adjoint(cfg: Config, U, Rbar, Ubar, ws=None, stream=None):
    """Ubar = (dR/dU)^T Rbar at U (overwrites Ubar)."""
    for t, n in ((U, "U"), (Rbar, "Rbar"), (Ubar, "Ubar")):
        _state(cfg, t, n)
    c = cfg.c_struct()
    _check(lib().rhs_adjoint(ctypes.byref(c), _ptr(U), _ptr(Rbar), _ptr(Ubar), _ptr(ws), _stream(stream)))
    return Ubar


def adjoint_workspace_bytes(cfg: Config) -> int:
    c = cfg.c_struct()
    out = ctypes.c_size_t(0)
    _check(lib().adjoint_workspace_bytes(ctypes.byref(c), ctypes.byref(out)))
    return out.value


def adjoint_workspace(cfg: Config, device="cuda") -> torch.Tensor:
    return torch.empty(adjoint_workspace_bytes(cfg), dtype=torch.uint8, device=device)


def rk3_step_adjoint(cfg: Config, Un: torch.Tensor, Ubar: torch.Tensor, dt: float, aws: torch.Tensor, stream=None):
    """In place: Ubar (cotangent of U^{n+1}) becomes the cotangent of U^n for one fixed-dt step from Un."""
    _state(cfg, Un, "Un")
    _state(cfg, Ubar, "Ubar")
    c = cfg.c_struct()
    _check(lib().rk3_step_adjoint(ctypes.byref(c), _ptr(Un), _ptr(Ubar), float(dt), _ptr(aws), _stream(stream)))
    return Ubar


def rk3_step_adjoint_stages(cfg: Config, Un: torch.Tensor, U1: torch.Tensor, U2: torch.Tensor, Ubar: torch.Tensor,
                            dt: float, aws: torch.Tensor, stream=None):
    """rk3_step_adjoint with the step's stage states U1, U2 given (as rk3_stage computes them)."""
    for t, n in ((Un, "Un"), (U1, "U1"), (U2, "U2"), (Ubar, "Ubar")):
        _state(cfg, t, n)
    c = cfg.c_struct()
    _check(lib().rk3_step_adjoint_stages(ctypes.byref(c), _ptr(Un), _ptr(U1), _ptr(U2), _ptr(Ubar), float(dt),
                                         _ptr(aws), _stream(stream)))
    return Ubar


def check_state(cfg: Config, U: torch.Tensor, ws: torch.Tensor, stream=None) -> Report:
    _state(cfg, U, "U")
    c = cfg.c_struct()
    rep = Report()
    code = lib().check_state(ctypes.byref(c), _ptr(U), _ptr(ws), ctypes.byref(rep), _stream(stream))
    if code not in (OK, EINADMISSIBLE, ENONFINITE):
        _check(code)
    return rep


def last_error() -> str:
    return lib().last_error().decode()


def config_from_case(case, dtype: int = F64, **over) -> Config:
    """Solver config for a workloads.Case."""
    kw = case.cfg_kwargs()
    kw.update(over)
    return Config(dtype=dtype, **kw)


def stage_workgroups(cfg: Config) -> int:
    """Workgroups of one fused stage launch of the problem."""
    c = cfg.c_struct()
    out = ctypes.c_int32(0)
    _check(lib().stage_workgroups(ctypes.byref(c), ctypes.byref(out)))
    return out.value


def workspace_time(cfg: Config, ws: torch.Tensor, stream=None) -> float:
    """Simulated time held in a workspace (synchronises the stream)."""
    c = cfg.c_struct()
    t = ctypes.c_double(0.0)
    _check(lib().workspace_time(ctypes.byref(c), _ptr(ws), ctypes.byref(t), _stream(stream)))
    return t.value


class Batch:
    """Handle of a batch of independent problems stepped together (``batch_*`` of the C ABI).

    The device request table is a tensor owned by this object; states and
    workspaces belong to the caller and must stay alive while they are members.
    """

    def __init__(self, capacity: int, device="cuda"):
        nb = ctypes.c_size_t(0)
        _check(lib().batch_table_bytes(int(capacity), ctypes.byref(nb)))
        self.capacity = int(capacity)
        self.table = torch.empty(nb.value, dtype=torch.uint8, device=device)
        h = ctypes.c_void_p(0)
        _check(lib().batch_create(self.capacity, _ptr(self.table), nb.value, ctypes.byref(h)))
        self._h = h
        self.members: list = []

    def set(self, members, fresh=None, stream=None):
        """members: sequence of (Config, U, ws); fresh: flags of members whose time stepping starts now."""
        n = len(members)
        cfgs = (_Cfg * max(1, n))()
        Us = (ctypes.c_void_p * max(1, n))()
        wss = (ctypes.c_void_p * max(1, n))()
        fr = (ctypes.c_int32 * max(1, n))()
        for i, (cfg, U, ws) in enumerate(members):
            _state(cfg, U, f"U[{i}]")
            if ws.numel() < workspace_bytes(cfg):
                raise ValueError(f"ws[{i}]: smaller than workspace_bytes")
            cfgs[i] = cfg.c_struct()
            Us[i] = _ptr(U)
            wss[i] = _ptr(ws)
            fr[i] = 1 if (fresh is not None and fresh[i]) else 0
        _check(lib().batch_set(self._h, n, cfgs, Us, wss, fr, _stream(stream)))
        self.members = list(members)

    def step(self, nsteps: int = 1, stream=None):
        _check(lib().batch_step(self._h, int(nsteps), _stream(stream)))

    def step_graph(self, nsteps: int = 1, stream=None):
        _check(lib().batch_step_graph(self._h, int(nsteps), _stream(stream)))

    def graph_count(self) -> int:
        """Step graphs cached by the batch (they survive membership changes)."""
        return lib().batch_graph_count(self._h)

    def close(self):
        if self._h is not None and self._h.value:
            _check(lib().batch_destroy(self._h))
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
