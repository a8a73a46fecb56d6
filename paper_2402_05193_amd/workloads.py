"""Seeded synthetic inputs shared by the HIP path and the oracle.

This module only builds initial *primitive* fields and problem descriptions; it
holds none of the scheme's arithmetic (no equation of state, no fluxes).  Each
side converts primitives to conservative variables with its own code.

Workloads (shapes and parameter values from the paper's test cases):

* Taylor-Green vortex on [0, 2pi)^3 with seeded uniform velocity noise
  (single-phase inviscid / Navier-Stokes benchmark case).
* Two-Gaussian density wave advected at u = p = 1 (Sec. 5.1, convergence test),
  initialised with exact cell averages.
* Planar two-state Riemann problems: the air-helium and air-water shock tubes
  (Sec. 5.3 tables) and seeded random ones.
* Three-dimensional air-helium shock-bubble interaction, Ma_S = 1.22
  (Sec. 5.3, shock-bubble tables), with the volume fraction smoothed by tanh.
* Uniform states and smooth random periodic fields (invariant checks).

Random numbers come from splitmix64 (Steele, Lea & Flood, OOPSLA 2014), keyed
by (seed, flat cell index, component), so every generator is reproducible
bit for bit on any machine.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

EULER, NS, DIM = 0, 1, 2
PERIODIC, ZERO_GRADIENT, SYMMETRY = 0, 1, 2

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """Output number (counter + 1) of a splitmix64 stream started at ``seed``."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (counters.astype(np.uint64) + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, counters: np.ndarray) -> np.ndarray:
    """53-bit uniform numbers in [0, 1)."""
    return (splitmix64(seed, counters) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def velocity_noise(seed: int, shape3, amplitude: float) -> np.ndarray:
    """Noise in [-amplitude, amplitude) for (u, v, w); counter = 3*flat_index + component."""
    n = int(np.prod(shape3))
    idx = np.arange(n, dtype=np.uint64)
    out = np.empty((3, n))
    for m in range(3):
        out[m] = amplitude * (2.0 * uniform01(seed, idx * np.uint64(3) + np.uint64(m)) - 1.0)
    return out.reshape((3,) + tuple(shape3))


@dataclass
class Case:
    """A problem: grid, model, boundary conditions, material and initial W."""
    name: str
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    model: int
    bc: tuple
    W: np.ndarray | None = None
    gamma1: float = 1.4
    pinf1: float = 0.0
    gamma2: float = 1.4
    pinf2: float = 0.0
    mu: float = 0.0
    prandtl: float = 0.72
    positivity: int = -1
    meta: dict = field(default_factory=dict)

    def cfg_kwargs(self) -> dict:
        """Keyword arguments accepted by both the oracle's and the solver's Config."""
        return dict(nx=self.nx, ny=self.ny, nz=self.nz, dx=self.dx, dy=self.dy, dz=self.dz,
                    model=self.model, bc=tuple(self.bc), gamma1=self.gamma1, pinf1=self.pinf1,
                    gamma2=self.gamma2, pinf2=self.pinf2, mu=self.mu, prandtl=self.prandtl,
                    positivity=self.positivity)


def _centres(n: int, h: float, x0: float = 0.0) -> np.ndarray:
    return x0 + (np.arange(n) + 0.5) * h


# --------------------------------------------------------------------------
# Taylor-Green vortex
# --------------------------------------------------------------------------
def taylor_green(n: int, ma: float = 0.1, gamma: float = 1.4, rho0: float = 1.0, noise: float = 1e-3,
                 seed: int = 2402, viscous: bool = False, reynolds: float = 1600.0,
                 prandtl: float = 0.72, ny: int | None = None, nz: int | None = None,
                 with_field: bool = True) -> Case:
    """rho = 1, u = sin x cos y cos z, v = -cos x sin y cos z, w = 0,
    p = 1/(gamma Ma^2) + (cos 2x + cos 2y)(cos 2z + 2)/16 on [0, 2pi)^3, plus
    seeded uniform +-noise on (u, v, w).  Viscous: mu = rho0 U0 L / Re with
    U0 = L = 1 (constant viscosity)."""
    ny = ny or n
    nz = nz or n
    h = 2.0 * math.pi / n
    case = Case(name=f"tgv{'_ns' if viscous else ''}_{n}x{ny}x{nz}", nx=n, ny=ny, nz=nz,
                dx=h, dy=2.0 * math.pi / ny, dz=2.0 * math.pi / nz,
                model=NS if viscous else EULER, bc=(PERIODIC,) * 6, gamma1=gamma,
                mu=(rho0 / reynolds if viscous else 0.0), prandtl=prandtl,
                meta=dict(ma=ma, seed=seed, noise=noise))
    if with_field:
        x = _centres(n, case.dx)[None, None, :]
        y = _centres(ny, case.dy)[None, :, None]
        z = _centres(nz, case.dz)[:, None, None]
        W = np.empty((5, nz, ny, n))
        W[0] = rho0
        W[1] = np.sin(x) * np.cos(y) * np.cos(z)
        W[2] = -np.cos(x) * np.sin(y) * np.cos(z)
        W[3] = 0.0
        W[4] = 1.0 / (gamma * ma * ma) + (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0) / 16.0
        if noise:
            W[1:4] += velocity_noise(seed, (nz, ny, n), noise)
        case.W = W
    return case


# --------------------------------------------------------------------------
# Convergence test: two Gaussians, exact cell averages (Sec. 5.1)
# --------------------------------------------------------------------------
def gauss_wave_density(n: int, length: float = 2.0) -> np.ndarray:
    """Cell averages of rho(x) = 1 + 5 exp(-200 (x-0.5)^2) + 5 exp(-200 (x-1.5)^2) on [0, length)."""
    h = length / n
    xf = np.arange(n + 1) * h
    s = math.sqrt(200.0)
    erf = np.vectorize(math.erf)
    # integral of 5 exp(-200 (x-c)^2) = 5 sqrt(pi)/(2 sqrt(200)) [erf(sqrt(200)(x-c))]
    total = np.zeros(n)
    for c in (0.5, 1.5):
        F = erf(s * (xf - c))
        total += 5.0 * math.sqrt(math.pi) / (2.0 * s) * (F[1:] - F[:-1])
    return 1.0 + total / h


def gauss_wave(n: int, axis: int = 0, gamma: float = 1.4) -> Case:
    """1-D density wave (u = 1 along ``axis``, p = 1) on a grid with n cells along
    ``axis`` and one cell in the other directions, periodic."""
    shape = [1, 1, 1]
    shape[axis] = n
    nx, ny, nz = shape
    h = 2.0 / n
    W = np.zeros((5, nz, ny, nx))
    rho = gauss_wave_density(n)
    view = [1, 1, 1]
    view[2 - axis] = n
    W[0] = rho.reshape(view)
    W[1 + axis] = 1.0
    W[4] = 1.0
    return Case(name=f"gauss_{'xyz'[axis]}_{n}", nx=nx, ny=ny, nz=nz, dx=h, dy=h, dz=h, model=EULER,
                bc=(PERIODIC,) * 6, W=W, gamma1=gamma)


def gauss_wave_diagonal(n: int, gamma: float = 1.4) -> Case:
    """The same profile advected along (1,1,1) on [0,2)^3 with velocity (1,1,1):
    density = product-free superposition along s = (x+y+z)/... is not separable,
    so cell averages use 3-point Gauss quadrature per direction of the
    one-dimensional profile evaluated at (x + y + z) mod 2."""
    h = 2.0 / n
    gx, gw = np.polynomial.legendre.leggauss(3)
    c = (np.arange(n) + 0.5) * h
    rho = np.zeros((n, n, n))

    def prof(s):
        s = np.mod(s, 2.0)
        out = 1.0
        for cc in (0.5, 1.5):
            for shift in (-2.0, 0.0, 2.0):
                out = out + 5.0 * np.exp(-200.0 * (s - cc + shift) ** 2)
        return out

    Z, Y, X = np.meshgrid(c, c, c, indexing="ij")
    for a, wa in zip(gx, gw):
        for b, wb in zip(gx, gw):
            for d, wd in zip(gx, gw):
                rho += wa * wb * wd / 8.0 * prof(X + a * h / 2 + Y + b * h / 2 + Z + d * h / 2)
    W = np.zeros((5, n, n, n))
    W[0] = rho
    W[1:4] = 1.0
    W[4] = 1.0
    return Case(name=f"gauss_diag_{n}", nx=n, ny=n, nz=n, dx=h, dy=h, dz=h, model=EULER,
                bc=(PERIODIC,) * 6, W=W, gamma1=gamma)


# --------------------------------------------------------------------------
# Uniform state and smooth random periodic fields
# --------------------------------------------------------------------------
def uniform(nx, ny, nz, model=EULER, state=(1.0, 0.1, -0.2, 0.3, 1.0), bc=(PERIODIC,) * 6,
            h=(0.1, 0.1, 0.1), **mat) -> Case:
    nc = 7 if model == DIM else 5
    W = np.empty((nc, nz, ny, nx))
    for m in range(nc):
        W[m] = state[m]
    return Case(name="uniform", nx=nx, ny=ny, nz=nz, dx=h[0], dy=h[1], dz=h[2], model=model, bc=bc, W=W,
                **mat)


def smooth_random(nx, ny, nz, model=EULER, seed=7, amplitude=0.2, bc=(PERIODIC,) * 6, h=None, **mat) -> Case:
    """Sum of a few seeded low Fourier modes per primitive, around a positive mean
    state, periodic on the box [0, 1)^3 (or the given spacing)."""
    nc = 7 if model == DIM else 5
    if h is None:
        h = (1.0 / nx, 1.0 / ny, 1.0 / nz)
    x = (np.arange(nx) + 0.5)[None, None, :] / nx
    y = (np.arange(ny) + 0.5)[None, :, None] / ny
    z = (np.arange(nz) + 0.5)[:, None, None] / nz
    if model == DIM:
        mean = [0.6, 0.5, 0.1, -0.1, 0.05, 1.0, 0.5]
    else:
        mean = [1.0, 0.2, -0.1, 0.15, 1.0]
    W = np.empty((nc, nz, ny, nx))
    cnt = np.arange(64, dtype=np.uint64)
    r = uniform01(seed, cnt)
    q = 0
    for m in range(nc):
        f = np.full((nz, ny, nx), mean[m])
        for _ in range(3):
            kx, ky, kz = 1 + int(3 * r[q % 64]), 1 + int(3 * r[(q + 1) % 64]), int(3 * r[(q + 2) % 64])
            ph = 2 * math.pi * r[(q + 3) % 64]
            amp = amplitude * abs(mean[m] if mean[m] != 0 else 1.0) * (0.5 + r[(q + 4) % 64]) / 3.0
            if m == (6 if model == DIM else -1):
                amp = 0.12
            f = f + amp * np.sin(2 * math.pi * (kx * x + ky * y + kz * z) + ph)
            q += 5
        W[m] = f
    return Case(name="smooth_random", nx=nx, ny=ny, nz=nz, dx=h[0], dy=h[1], dz=h[2], model=model, bc=bc,
                W=W, **mat)


# --------------------------------------------------------------------------
# Riemann problems
# --------------------------------------------------------------------------
def riemann_planar(nx, ny, nz, axis, x0_frac, WL, WR, model, h, bc=(ZERO_GRADIENT,) * 6, **mat) -> Case:
    """Two constant primitive states separated by the plane at x0_frac of the
    domain length along ``axis``."""
    nc = 7 if model == DIM else 5
    n = (nx, ny, nz)[axis]
    c = (np.arange(n) + 0.5) / n
    left = c < x0_frac
    shape = [1, 1, 1]
    shape[2 - axis] = n
    mask = left.reshape(shape)
    W = np.empty((nc, nz, ny, nx))
    for m in range(nc):
        W[m] = np.where(mask, WL[m], WR[m])
    return Case(name="riemann", nx=nx, ny=ny, nz=nz, dx=h, dy=h, dz=h, model=model, bc=bc, W=W, **mat)


ALPHA_EPS = 1e-8   # volume fraction in the "pure" phases (Sec. 5.3)


def air_helium_tube(n: int = 200) -> Case:
    """Air (x <= 0.5: rho 1, p 1, gamma 1.4) | helium (rho 0.125, p 0.1, gamma 1.67), zero-gradient ends.
    Fluid 1 = air, fluid 2 = helium."""
    a = 1.0 - ALPHA_EPS
    WL = (a * 1.0, (1 - a) * 0.125, 0.0, 0.0, 0.0, 1.0, a)
    b = ALPHA_EPS
    WR = (b * 1.0, (1 - b) * 0.125, 0.0, 0.0, 0.0, 0.1, b)
    case = riemann_planar(n, 1, 1, 0, 0.5, WL, WR, DIM, 1.0 / n, gamma1=1.4, gamma2=1.67)
    case.name = f"air_helium_{n}"
    case.meta = dict(t_end=0.15, left=(1.0, 0.0, 1.0, 1.4, 0.0), right=(0.125, 0.0, 0.1, 1.67, 0.0), x0=0.5,
                     length=1.0)
    return case


def air_water_tube(n: int = 200, t_end: float = 1.5e-4) -> Case:
    """Water (x <= 0.8: rho 1000, p 1e9, gamma 6.12, pinf 3.43e8) | air (rho 20, p 1e5, gamma 1.4)
    on [0, 1.5] with zero-gradient ends.  Fluid 1 = water, fluid 2 = air."""
    a = 1.0 - ALPHA_EPS
    b = ALPHA_EPS
    WL = (a * 1000.0, (1 - a) * 20.0, 0.0, 0.0, 0.0, 1e9, a)
    WR = (b * 1000.0, (1 - b) * 20.0, 0.0, 0.0, 0.0, 1e5, b)
    case = riemann_planar(n, 1, 1, 0, 0.8 / 1.5, WL, WR, DIM, 1.5 / n, gamma1=6.12, pinf1=3.43e8,
                          gamma2=1.4, pinf2=0.0)
    case.name = f"air_water_{n}"
    case.meta = dict(t_end=t_end, left=(1000.0, 0.0, 1e9, 6.12, 3.43e8), right=(20.0, 0.0, 1e5, 1.4, 0.0),
                     x0=0.8, length=1.5)
    return case


def sod_tube(n: int = 200) -> Case:
    WL = (1.0, 0.0, 0.0, 0.0, 1.0)
    WR = (0.125, 0.0, 0.0, 0.0, 0.1)
    case = riemann_planar(n, 1, 1, 0, 0.5, WL, WR, EULER, 1.0 / n, gamma1=1.4)
    case.name = f"sod_{n}"
    case.meta = dict(t_end=0.2, left=(1.0, 0.0, 1.0, 1.4, 0.0), right=(0.125, 0.0, 0.1, 1.4, 0.0), x0=0.5,
                     length=1.0)
    return case


# --------------------------------------------------------------------------
# Shock-bubble interaction
# --------------------------------------------------------------------------
def interface_advection(n: int = 48, axis: int = 0, flip: bool = False, u: float = 0.5) -> Case:
    """Two smeared helium/air interfaces (tanh profiles a few cells wide) in a
    periodic line along `axis`, advected at uniform velocity and pressure: the
    five-equation model with an interface band of about eight cells
    (volume fraction between 1e-6 and 1 - 1e-6).  `flip` mirrors the field and
    the velocity."""
    shape = [1, 1, 1]
    shape[2 - axis] = n
    x = (np.arange(n) + 0.5) / n
    a = 0.5 * (1 + np.tanh((x - 0.3) * n / 2.0)) * 0.5 * (1 - np.tanh((x - 0.7) * n / 2.0))
    a = 1e-6 + (1 - 2e-6) * a
    if flip:
        a = a[::-1].copy()
    W = np.zeros((7, *shape))
    r1, r2 = 0.166, 1.2
    W[0] = (a * r1).reshape(shape)
    W[1] = ((1 - a) * r2).reshape(shape)
    W[2 + axis] = -u if flip else u
    W[5] = 1.0
    W[6] = a.reshape(shape)
    h = 1.0 / n
    return Case(name=f"interface_{'xyz'[axis]}_{n}", nx=shape[2], ny=shape[1], nz=shape[0], dx=h, dy=h, dz=h,
                model=DIM, bc=(PERIODIC,) * 6, W=W, gamma1=1.66, gamma2=1.4, positivity=1)


def rankine_hugoniot(ma: float, gamma: float, rho1: float, p1: float, pinf: float = 0.0):
    """Post-shock (rho2, u2, p2) behind a shock of Mach number ma moving into
    fluid at rest (rho1, p1), stiffened gas; returns (rho2, u2, p2, shock_speed)."""
    c1 = math.sqrt(gamma * (p1 + pinf) / rho1)
    us = ma * c1
    m2 = ma * ma
    p2 = p1 + (p1 + pinf) * 2.0 * gamma / (gamma + 1.0) * (m2 - 1.0)
    rho2 = rho1 * (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    u2 = us * (1.0 - rho1 / rho2)
    return rho2, u2, p2, us


def shock_bubble(nx: int = 256, ny: int = 128, nz: int = 128, ma: float = 1.22, gamma_he: float = 1.66,
                 with_field: bool = True) -> Case:
    """Air (fluid 2, gamma 1.4) at rest, a Ma_S planar shock at x = 60 mm moving +x into a
    helium sphere (fluid 1) of radius 0.25 H centred at (90 mm, H/2, H/2); H = 89 mm,
    domain [0, 2H] x [0, H] x [0, H]; volume fraction smoothed with tanh over two cells;
    zero-gradient boundaries.  SI units."""
    H = 0.089
    L = 2.0 * H
    h = L / nx
    rho_air, p_air = 1.2041, 101325.0
    rho_he = 0.1660
    rho2, u2, p2, us = rankine_hugoniot(ma, 1.4, rho_air, p_air)
    case = Case(name=f"sbi_{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, dx=h, dy=H / ny, dz=H / nz, model=DIM,
                bc=(ZERO_GRADIENT,) * 6, gamma1=gamma_he, gamma2=1.4, positivity=1,
                meta=dict(ma=ma, post_shock=(rho2, u2, p2), shock_speed=us, H=H))
    if with_field:
        x = _centres(nx, case.dx)[None, None, :]
        y = _centres(ny, case.dy)[None, :, None]
        z = _centres(nz, case.dz)[:, None, None]
        r = np.sqrt((x - 0.090) ** 2 + (y - H / 2) ** 2 + (z - H / 2) ** 2)
        R = 0.25 * H
        eps = ALPHA_EPS
        a1 = eps + (1.0 - 2.0 * eps) * 0.5 * (1.0 - np.tanh((r - R) / h))
        shocked = np.broadcast_to(x < 0.060, r.shape)
        rho_a = np.where(shocked, rho2, rho_air)
        u = np.where(shocked, u2, 0.0)
        p = np.where(shocked, p2, p_air)
        W = np.empty((7, nz, ny, nx))
        W[0] = a1 * rho_he
        W[1] = (1.0 - a1) * rho_a
        W[2] = u
        W[3] = 0.0
        W[4] = 0.0
        W[5] = p
        W[6] = a1
        case.W = W
    return case


# --------------------------------------------------------------------------
# Serving workload: a stream of independent three-dimensional Riemann problems
# --------------------------------------------------------------------------
SERVING_GRIDS = ((64, 64, 64), (96, 96, 96), (128, 128, 128), (192, 96, 96), (256, 128, 128))


@dataclass
class RiemannRequest:
    """One request of the serving stream: a planar Riemann problem normal to x
    at mid-domain in a box of cubic cells (h = 1/nx, domain [0,1] x [0,ny h] x
    [0,nz h]), zero-gradient boundaries, tangential velocity 0.  Two-phase
    requests carry fluid 1 (gamma 1.4) on the left and fluid 2 (gamma 1.66) on
    the right with volume fractions 1 - ALPHA_EPS / ALPHA_EPS."""
    index: int
    model: int
    nx: int
    ny: int
    nz: int
    h: float
    WL: tuple
    WR: tuple
    left: tuple    # (rho, u, p, gamma) for an exact solution
    right: tuple
    gamma1: float
    gamma2: float
    steps: int

    @property
    def ncells(self) -> int:
        return self.nx * self.ny * self.nz

    def cfg_kwargs(self) -> dict:
        return dict(nx=self.nx, ny=self.ny, nz=self.nz, dx=self.h, dy=self.h, dz=self.h, model=self.model,
                    bc=(ZERO_GRADIENT,) * 6, gamma1=self.gamma1, gamma2=self.gamma2, positivity=1)

    def riemann_params(self) -> list:
        """Parameters of the planar two-state initial condition: axis, x0 fraction, W_L, W_R."""
        return [0.0, 0.5, *self.WL, *self.WR]


def riemann_request(index: int, seed: int = 2402, grids=SERVING_GRIDS, steps: int = 50,
                    two_phase_fraction: float = 0.5) -> RiemannRequest:
    """Request number ``index`` of the serving stream (seeded, reproducible).

    rho in [0.1, 10], p in [0.1, 10], normal velocity in [-1, 1] on each side,
    uniform draws.  Draws that would open a vacuum (u_R - u_L at or above
    2 c_L/(gamma_L - 1) + 2 c_R/(gamma_R - 1)) are redrawn."""
    attempt = 0
    while True:
        ctr = np.arange(16, dtype=np.uint64) + np.uint64(16 * (index * 64 + attempt))
        u = uniform01(seed, ctr)
        g = grids[min(int(u[0] * len(grids)), len(grids) - 1)]
        model = DIM if u[1] < two_phase_fraction else EULER
        u = [float(x) for x in u]
        rl, rr = 0.1 + 9.9 * u[2], 0.1 + 9.9 * u[3]
        pl, pr = 0.1 + 9.9 * u[4], 0.1 + 9.9 * u[5]
        ul, ur = -1.0 + 2.0 * u[6], -1.0 + 2.0 * u[7]
        gl, gr = (1.4, 1.66) if model == DIM else (1.4, 1.4)
        cl, cr = math.sqrt(gl * pl / rl), math.sqrt(gr * pr / rr)
        if 2 * cl / (gl - 1) + 2 * cr / (gr - 1) > (ur - ul):
            break
        attempt += 1
    if model == DIM:
        a, b = 1.0 - ALPHA_EPS, ALPHA_EPS
        WL = (a * rl, (1 - a) * rl, ul, 0.0, 0.0, pl, a)
        WR = (b * rr, (1 - b) * rr, ur, 0.0, 0.0, pr, b)
    else:
        WL = (rl, ul, 0.0, 0.0, pl)
        WR = (rr, ur, 0.0, 0.0, pr)
    nx, ny, nz = g
    return RiemannRequest(index=index, model=model, nx=nx, ny=ny, nz=nz, h=1.0 / nx, WL=WL, WR=WR,
                          left=(rl, ul, pl, gl), right=(rr, ur, pr, gr), gamma1=1.4,
                          gamma2=1.66 if model == DIM else 1.4, steps=steps)


def poisson_arrivals(n: int, rate: float, seed: int = 2402) -> np.ndarray:
    """Arrival times (s) of the first n events of a Poisson process of the given rate."""
    u = uniform01(seed ^ 0x5EED, np.arange(n, dtype=np.uint64))
    return np.cumsum(-np.log1p(-u) / rate)


# --------------------------------------------------------------------------
# Differentiation workload: compressible decaying turbulence
# --------------------------------------------------------------------------
def decaying_turbulence(n: int, seed: int = 0, urms: float = 0.3, k0: float = 4.0, gamma: float = 1.4):
    """Primitive state of compressible decaying turbulence on [0, 2pi)^3: rho = 1,
    p = 1/gamma, solenoidal velocity with random phases and energy spectrum
    E(k) ~ k^4 exp(-2 (k/k0)^2), scaled to u_rms = sqrt(<u.u>/3) = urms.
    Seeded; built with an FFT on the host."""
    k1 = np.fft.fftfreq(n, d=1.0 / n)
    KZ, KY, KX = np.meshgrid(k1, k1, k1, indexing="ij")
    K = np.sqrt(KX ** 2 + KY ** 2 + KZ ** 2)
    ctr = np.arange(6 * n ** 3, dtype=np.uint64).reshape(6, n, n, n)
    u = uniform01(seed, ctr)
    # complex Gaussian amplitudes (Box-Muller), one per component
    r = np.sqrt(-2.0 * np.log1p(-u[0:3]))
    ph = 2.0 * math.pi * u[3:6]
    A = r * np.exp(1j * ph)
    # project out the component along k (divergence-free), shape by the spectrum
    Kn = np.where(K > 0, K, 1.0)
    kv = np.stack([KX, KY, KZ]) / Kn
    A = A - kv * (kv * A).sum(0)
    amp = np.where(K > 0, K ** 2 * np.exp(-((K / k0) ** 2)) / Kn, 0.0)   # |u_k| ~ sqrt(E(k)/k^2)
    vel = np.real(np.fft.ifftn(A * amp, axes=(1, 2, 3)))
    vel -= vel.mean(axis=(1, 2, 3), keepdims=True)
    vel *= urms / math.sqrt((vel ** 2).sum(0).mean() / 3.0)
    W = np.empty((5, n, n, n))
    W[0] = 1.0
    W[1], W[2], W[3] = vel[0], vel[1], vel[2]
    W[4] = 1.0 / gamma
    return W
