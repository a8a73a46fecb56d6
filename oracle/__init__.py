"""FP64 CPU oracle of the finite-volume RHS / TVD-RK3 path (test infrastructure).

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It loads ``oracle/liboracle.so`` (plain
C, built by ``oracle/Makefile``) and shares no code with the HIP library.

Every array is numpy float64 in structure-of-arrays layout
``[ncomp, nz, ny, nx]``.  Component order follows the paper's state vectors:
single phase ``U = (rho, rho u, rho v, rho w, E)``, ``W = (rho, u, v, w, p)``;
five-equation model ``U = (a1 rho1, a2 rho2, rho u, rho v, rho w, E, a1)``,
``W = (a1 rho1, a2 rho2, u, v, w, p, a1)`` (Sec. 2.1 and 2.3).
"""
from __future__ import annotations

import contextlib
import ctypes
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

EULER, NS, DIM = 0, 1, 2
PERIODIC, ZERO_GRADIENT, SYMMETRY = 0, 1, 2

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_FMA_PATH = os.path.join(_HERE, "liboracle_fma.so")
_ULP_PATH = os.path.join(_HERE, "liboracle_ulp.so")
_lib = None
_variants = {}


def build() -> None:
    """Compile liboracle.so with the oracle's own Makefile, and the same source with
    multiply-add contraction (liboracle_fma.so, used only to calibrate round-off floors)."""
    subprocess.run(["make", "-s", "-C", _HERE, "-B", "liboracle.so"], check=True)
    subprocess.run(["make", "-s", "-C", _HERE, "-B", "fma", f"FMA_OUT={_FMA_PATH}"], check=True)
    subprocess.run(["make", "-s", "-C", _HERE, "-B", "ulp", f"ULP_OUT={_ULP_PATH}"], check=True)


class _Cfg(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("model", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 6),
        ("positivity", ctypes.c_int32), ("recon", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("dz", ctypes.c_double),
        ("gamma1", ctypes.c_double), ("pinf1", ctypes.c_double),
        ("gamma2", ctypes.c_double), ("pinf2", ctypes.c_double),
        ("mu", ctypes.c_double), ("prandtl", ctypes.c_double),
        ("eps_rho", ctypes.c_double), ("eps_rhoc2", ctypes.c_double), ("eps_alpha", ctypes.c_double),
        ("weno_eps", ctypes.c_double),
        ("visc_law", ctypes.c_int32), ("scheme", ctypes.c_int32),
        ("T_ref", ctypes.c_double), ("sutherland", ctypes.c_double), ("gas_R", ctypes.c_double),
        ("visc_order", ctypes.c_int32), ("thinc", ctypes.c_int32),
    ]


@dataclass
class Config:
    """Problem description (grid, model, boundary conditions, material)."""
    nx: int
    ny: int
    nz: int
    dx: float = 1.0
    dy: float = 1.0
    dz: float = 1.0
    model: int = EULER
    bc: tuple = (PERIODIC,) * 6
    gamma1: float = 1.4
    pinf1: float = 0.0
    gamma2: float = 1.4
    pinf2: float = 0.0
    mu: float = 0.0
    prandtl: float = 0.72
    positivity: int = -1          # -1: on for the five-equation model, off otherwise
    eps_rho: float = 1e-12        # FP64 tolerances of Sec. 3.3
    eps_rhoc2: float = 1e-10
    eps_alpha: float = 1e-12
    weno_eps: float = 1e-40
    recon: int = 0                # 0: primitive variables, 1: characteristic variables
    visc_law: int = 0             # 0: constant mu, 1: power law, 2: Sutherland (Sec. 2.5)
    scheme: int = 0               # 0: WENO5-Z, 1: TENO6-A (Sec. 3.2 step 3)
    visc_order: int = 4           # central viscous stencils: 4th or 6th order
    thinc: int = 0                # 1: THINC volume-fraction faces in interface cells (DIM)
    T_ref: float = 1.0
    sutherland: float = 0.0
    gas_R: float = 1.0

    @property
    def ncomp(self) -> int:
        return 7 if self.model == DIM else 5

    @property
    def shape(self):
        return (self.ncomp, self.nz, self.ny, self.nx)

    def c_struct(self) -> _Cfg:
        c = _Cfg()
        c.nx, c.ny, c.nz = self.nx, self.ny, self.nz
        c.model = self.model
        for i, b in enumerate(self.bc):
            c.bc[i] = int(b)
        pos = self.positivity
        if pos < 0:
            pos = 1 if self.model == DIM else 0
        c.positivity = pos
        c.dx, c.dy, c.dz = self.dx, self.dy, self.dz
        c.gamma1, c.pinf1, c.gamma2, c.pinf2 = self.gamma1, self.pinf1, self.gamma2, self.pinf2
        c.mu, c.prandtl = self.mu, self.prandtl
        c.eps_rho, c.eps_rhoc2, c.eps_alpha = self.eps_rho, self.eps_rhoc2, self.eps_alpha
        c.weno_eps = self.weno_eps
        c.recon = self.recon
        c.visc_law = self.visc_law
        c.scheme = self.scheme
        c.visc_order = self.visc_order
        c.thinc = self.thinc
        c.T_ref, c.sutherland, c.gas_R = self.T_ref, self.sutherland, self.gas_R
        return c


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        _lib = _load(_LIB_PATH)
    return _lib


@contextlib.contextmanager
def variant(kind: str):
    """Within the block every oracle call runs a calibration build of the same
    source: kind "fma" -- multiply-add contraction (every intermediate rounded
    differently, which a one-ulp move of the input does not reach); kind "ulp" --
    every exp, pow, tanh, atanh, cosh and sinh result one unit in the last place
    higher (another correct math library's rounding).  Their differences from the
    reference build are the oracle's own round-off floor."""
    global _lib
    path, target, var = {"fma": (_FMA_PATH, "fma", "FMA_OUT"), "ulp": (_ULP_PATH, "ulp", "ULP_OUT")}[kind]
    saved = lib()
    if kind not in _variants:
        if not os.path.exists(path):
            subprocess.run(["make", "-s", "-C", _HERE, "-B", target, f"{var}={path}"], check=True)
        _variants[kind] = _load(path)
    _lib = _variants[kind]
    try:
        yield
    finally:
        _lib = saved


def contracted():
    """variant("fma")."""
    return variant("fma")


def _load(path):
    """Load one build of the oracle and declare its entry points."""
    L = ctypes.CDLL(path)
    dp = ctypes.POINTER(ctypes.c_double)
    cp = ctypes.POINTER(_Cfg)
    L.orc_ncomp.argtypes = [cp]
    L.orc_prim_to_cons.argtypes = [cp, dp, dp]
    L.orc_cons_to_prim.argtypes = [cp, dp, dp]
    L.orc_weno5z.argtypes = [ctypes.c_double] * 6
    L.orc_weno5z.restype = ctypes.c_double
    L.orc_teno6a_parts.argtypes = [dp, ctypes.c_double, dp]
    L.orc_teno6a_parts.restype = ctypes.c_double
    L.orc_thinc_faces.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double, dp]
    L.orc_hllc.argtypes = [cp, ctypes.c_int, dp, dp, dp, dp]
    L.orc_rhs.argtypes = [cp, dp, dp, ctypes.c_double, ctypes.POINTER(ctypes.c_uint8)]
    L.orc_rhs_cells.argtypes = [cp, dp, ctypes.POINTER(ctypes.c_int64), ctypes.c_int64, dp, ctypes.c_double,
                                ctypes.POINTER(ctypes.c_uint8)]
    L.orc_hllc_speeds.argtypes = [cp, ctypes.c_int, dp, dp, dp, dp]
    L.orc_thinc_beta.argtypes = [dp, dp, ctypes.c_int]
    L.orc_thinc_beta.restype = ctypes.c_double
    L.orc_rk3_stage.argtypes = [cp, ctypes.c_int, dp, dp, dp, ctypes.c_double]
    L.orc_dt.argtypes = [cp, dp, ctypes.c_double]
    L.orc_dt.restype = ctypes.c_double
    L.orc_advance.argtypes = [cp, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double]
    L.orc_advance.restype = ctypes.c_double
    L.orc_char_matrices.argtypes = [cp, ctypes.c_int, dp, dp, dp]
    L.orc_face_count.argtypes = [cp, ctypes.c_int]
    L.orc_face_count.restype = ctypes.c_long
    L.orc_max_threads.restype = ctypes.c_int
    L.orc_set_threads.argtypes = [ctypes.c_int]
    return L


def _dp(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _arr(a, shape=None) -> np.ndarray:
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def prim_to_cons(cfg: Config, W) -> np.ndarray:
    W = _arr(W, cfg.shape)
    U = np.empty_like(W)
    c = cfg.c_struct()
    lib().orc_prim_to_cons(ctypes.byref(c), _dp(W), _dp(U))
    return U


def cons_to_prim(cfg: Config, U) -> np.ndarray:
    U = _arr(U, cfg.shape)
    W = np.empty_like(U)
    c = cfg.c_struct()
    lib().orc_cons_to_prim(ctypes.byref(c), _dp(U), _dp(W))
    return W


def weno5z(a, b, c, d, e, eps=1e-40) -> float:
    return lib().orc_weno5z(a, b, c, d, e, eps)


def thinc_faces(abar, theta, beta):
    """THINC profile of a cell with mean abar: (value at the -d face, value at the
    +d face, interface centre x_c)."""
    out = np.zeros(3)
    lib().orc_thinc_faces(float(abar), float(theta), float(beta), _dp(out))
    return tuple(out)


TENO_PARTS = ("beta0", "beta1", "beta2", "beta3", "beta6", "tau6", "CT", "delta0", "delta1", "delta2", "delta3",
              "omega0", "omega1", "omega2", "omega3")


def teno6a(v, eps=1e-40, parts=False):
    """Left-biased TENO6-A value at x_{i+1/2} from v_{i-2..i+3}; with parts, also
    the intermediate quantities named in TENO_PARTS."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    assert v.shape == (6,)
    out = np.zeros(len(TENO_PARTS))
    val = lib().orc_teno6a_parts(_dp(v), eps, _dp(out))
    if parts:
        return val, dict(zip(TENO_PARTS, out))
    return val


def hllc(cfg: Config, d: int, WL, WR):
    """HLLC flux (global frame) and upwinded normal velocity at a face normal to d."""
    WL = _arr(WL)
    WR = _arr(WR)
    F = np.empty(cfg.ncomp)
    uh = np.zeros(1)
    c = cfg.c_struct()
    lib().orc_hllc(ctypes.byref(c), d, _dp(WL), _dp(WR), _dp(F), _dp(uh))
    return F, float(uh[0])


def hllc_speeds(cfg: Config, d: int, WL, WR):
    """Einfeldt signal speeds (s_L, s_R) the HLLC flux uses at a face normal to d."""
    WL = _arr(WL)
    WR = _arr(WR)
    sl = np.zeros(1)
    sr = np.zeros(1)
    c = cfg.c_struct()
    lib().orc_hllc_speeds(ctypes.byref(c), d, _dp(WL), _dp(WR), _dp(sl), _dp(sr))
    return float(sl[0]), float(sr[0])


def thinc_beta(a6, h, d: int) -> float:
    """beta_i of THINC along d from the volume fractions of the six face neighbours
    (-x, +x, -y, +y, -z, +z) and the cell sizes h (Sec. 3.2 and 3.7)."""
    a6 = _arr(a6, (6,))
    h = _arr(h, (3,))
    return lib().orc_thinc_beta(_dp(a6), _dp(h), int(d))


def face_counts(cfg: Config):
    c = cfg.c_struct()
    return [lib().orc_face_count(ctypes.byref(c), d) for d in range(3)]


def rhs(cfg: Config, U, dt: float = 0.0, return_flags: bool = False):
    """R_NSE(U) (Eq. FVD + DIM source).  dt is used only by the flux limiter."""
    U = _arr(U, cfg.shape)
    R = np.empty_like(U)
    c = cfg.c_struct()
    flags = None
    fptr = None
    if return_flags:
        flags = np.zeros(sum(face_counts(cfg)), dtype=np.uint8)
        fptr = flags.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    lib().orc_rhs(ctypes.byref(c), _dp(U), _dp(R), float(dt), fptr)
    if return_flags:
        out = []
        off = 0
        for d, nf in enumerate(face_counts(cfg)):
            shp = [cfg.nz, cfg.ny, cfg.nx]
            shp[2 - d] += 1
            out.append(flags[off:off + nf].reshape(shp))
            off += nf
        return R, out
    return R


def rhs_cells(cfg: Config, U, cells, dt: float = 0.0, return_flags: bool = False):
    """R at the given flat cell indices, shape [ncomp, len(cells)]; with
    return_flags also the limiter decisions of each cell's six faces, shape
    [len(cells), 6] in the order -x, +x, -y, +y, -z, +z."""
    U = _arr(U, cfg.shape)
    cells = np.ascontiguousarray(cells, dtype=np.int64)
    out = np.empty((cfg.ncomp, len(cells)))
    flags = np.zeros((len(cells), 6), dtype=np.uint8) if return_flags else None
    fptr = flags.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) if return_flags else None
    c = cfg.c_struct()
    lib().orc_rhs_cells(ctypes.byref(c), _dp(U), cells.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                        len(cells), _dp(out), float(dt), fptr)
    return (out, flags) if return_flags else out


def rk3_stage(cfg: Config, stage: int, Un, Uk, dt: float) -> np.ndarray:
    Un = _arr(Un, cfg.shape)
    Uk = _arr(Uk, cfg.shape)
    out = np.empty_like(Un)
    c = cfg.c_struct()
    lib().orc_rk3_stage(ctypes.byref(c), stage, _dp(Un), _dp(Uk), _dp(out), float(dt))
    return out


def rk3_step(cfg: Config, U, dt: float) -> np.ndarray:
    U1 = rk3_stage(cfg, 1, U, U, dt)
    U2 = rk3_stage(cfg, 2, U, U1, dt)
    return rk3_stage(cfg, 3, U, U2, dt)


def compute_dt(cfg: Config, U, cfl: float) -> float:
    U = _arr(U, cfg.shape)
    c = cfg.c_struct()
    return lib().orc_dt(ctypes.byref(c), _dp(U), float(cfl))


def advance(cfg: Config, U, nsteps: int, dt: float = 0.0, cfl: float = 0.5):
    """Advance nsteps (fixed dt if dt > 0, else CFL).  Returns (U, t)."""
    U = _arr(U, cfg.shape).copy()
    c = cfg.c_struct()
    t = lib().orc_advance(ctypes.byref(c), _dp(U), int(nsteps), float(dt), float(cfl))
    return U, t


def char_matrices(cfg: Config, d: int, W):
    """Right eigenvectors K (columns) of A(W) for direction d and K^{-1} (Sec. 3.2, appendix)."""
    nc = cfg.ncomp
    W = _arr(W, (nc,))
    K = np.zeros((nc, nc))
    Ki = np.zeros((nc, nc))
    c = cfg.c_struct()
    lib().orc_char_matrices(ctypes.byref(c), int(d), _dp(W), _dp(K), _dp(Ki))
    return K, Ki


def max_threads() -> int:
    return lib().orc_max_threads()


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))
