"""Plain PyTorch (CPU, FP64) right-hand side of the single-phase Euler equations
and its exact vector-Jacobian product, the reference of the discrete adjoint.

TEST INFRASTRUCTURE ONLY: used by the test suite; the HIP library never loads
it and shares no code with it.

The right-hand side is the finite-volume discretisation of arXiv:2402.05193
(Eq. (FVD), Sec. 3.2) for the inviscid single-phase model (Sec. 2.1, stiffened
gas of Sec. 2.4): boundary conditions by halo fill (Sec. 3.1), primitive
variables, WENO5-Z reconstruction of each primitive component on both sides of
every face (Sec. 3.2 step 3), HLLC flux with Einfeldt / Batten speeds
(Sec. 3.2 step 6 and the HLLC appendix), flux divergence.  The readings are
those of the C oracle (q = 1, d = 1/10 on {i-2, i-1, i}, Roe averages in the
Einfeldt speeds, sgn(0) = 0).  Whole arrays are processed at once with torch
operations, so torch.autograd gives the exact derivative of this discrete
operator: the adjoint (dR/dU)^T Rbar is one backward pass (Sec. 6, automatic
differentiation of the solver).  Where the operator is not differentiable
(|x| at 0, min/max at ties, the sgn switch of the HLLC flux) the derivative is
the one torch assigns: 0 for |x|' and for the switch, the even split at a tie
of min/max.

The TVD-RK3 step (Sec. 3.4) at a fixed dt is built from it.
"""
from __future__ import annotations

import numpy as np
import torch

PERIODIC, ZERO_GRADIENT, SYMMETRY = 0, 1, 2
H = 3  # halo width of WENO5


def _map_index(n: int, lo: int, hi: int):
    """Interior index and momentum sign of padded positions -H .. n+H-1 along one axis."""
    idx = np.empty(n + 2 * H, dtype=np.int64)
    sign = np.ones(n + 2 * H)
    for p in range(n + 2 * H):
        g = p - H
        s = 1.0
        if g < 0:
            if lo == PERIODIC:
                g = g % n
            elif lo == ZERO_GRADIENT:
                g = 0
            else:
                g = min(-g - 1, n - 1)
                s = -1.0
        elif g >= n:
            if hi == PERIODIC:
                g = g % n
            elif hi == ZERO_GRADIENT:
                g = n - 1
            else:
                g = max(2 * n - 1 - g, 0)
                s = -1.0
        idx[p] = g
        sign[p] = s
    return torch.from_numpy(idx), torch.from_numpy(sign)


def pad(cfg, U: torch.Tensor) -> torch.Tensor:
    """Conservative state with a 3-cell halo on every side (Sec. 3.1)."""
    ix, sx = _map_index(cfg.nx, cfg.bc[0], cfg.bc[1])
    iy, sy = _map_index(cfg.ny, cfg.bc[2], cfg.bc[3])
    iz, sz = _map_index(cfg.nz, cfg.bc[4], cfg.bc[5])
    P = U[:, iz][:, :, iy][:, :, :, ix]
    flips = [sx.view(1, 1, -1), sy.view(1, -1, 1), sz.view(-1, 1, 1)]
    rows = [P[0]] + [P[1 + d] * flips[d] for d in range(3)] + [P[4]]
    return torch.stack(rows)


def cons_to_prim(cfg, U):
    """W = (rho, u, v, w, p) from U = (rho, rho u, rho v, rho w, E), stiffened gas (Sec. 2.4)."""
    g, pinf = cfg.gamma1, cfg.pinf1
    rho = U[0]
    vel = [U[1 + d] / rho for d in range(3)]
    ke = 0.5 * rho * (vel[0] * vel[0] + vel[1] * vel[1] + vel[2] * vel[2])
    p = (g - 1.0) * (U[4] - ke) - g * pinf
    return [rho, vel[0], vel[1], vel[2], p]


def weno5z(a, b, c, d, e, eps):
    """WENO5-Z value at x_{i+1/2} from v_{i-2} .. v_{i+2} (Sec. 3.2 step 3; q = 1)."""
    p0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0
    p1 = (-b + 5.0 * c + 2.0 * d) / 6.0
    p2 = (2.0 * c + 5.0 * d - e) / 6.0
    b0 = 13.0 / 12.0 * (a - 2.0 * b + c) ** 2 + 0.25 * (a - 4.0 * b + 3.0 * c) ** 2
    b1 = 13.0 / 12.0 * (b - 2.0 * c + d) ** 2 + 0.25 * (b - d) ** 2
    b2 = 13.0 / 12.0 * (c - 2.0 * d + e) ** 2 + 0.25 * (3.0 * c - 4.0 * d + e) ** 2
    tau = torch.abs(b0 - b2)
    a0 = 0.1 * (1.0 + tau / (b0 + eps))
    a1 = 0.6 * (1.0 + tau / (b1 + eps))
    a2 = 0.3 * (1.0 + tau / (b2 + eps))
    s = a0 + a1 + a2
    return (a0 / s) * p0 + (a1 / s) * p1 + (a2 / s) * p2


def hllc(cfg, d, WL, WR):
    """HLLC flux normal to axis d between primitive states WL, WR (lists of arrays)."""
    g, pinf = cfg.gamma1, cfg.pinf1
    rL, rR = WL[0], WR[0]
    uL, uR = WL[1 + d], WR[1 + d]
    pL, pR = WL[4], WR[4]
    cL = torch.sqrt(g * (pL + pinf) / rL)
    cR = torch.sqrt(g * (pR + pinf) / rR)
    sqL, sqR = torch.sqrt(rL), torch.sqrt(rR)
    ubar = (sqL * uL + sqR * uR) / (sqL + sqR)
    cbar2 = (sqL * cL * cL + sqR * cR * cR) / (sqL + sqR) + 0.5 * sqL * sqR / ((sqL + sqR) ** 2) * (uR - uL) ** 2
    cbar = torch.sqrt(cbar2)
    sL = torch.minimum(ubar - cbar, uL - cL)
    sR = torch.maximum(ubar + cbar, uR + cR)
    zero = torch.zeros_like(sL)
    sminus = torch.minimum(zero, sL)
    splus = torch.maximum(zero, sR)
    tL, tR = rL * uL * (sL - uL), rR * uR * (sR - uR)
    sstar = ((pR - pL) + (tL - tR)) / (rL * (sL - uL) - rR * (sR - uR))

    def state(W, s, u):
        rho, p = W[0], W[4]
        E = (p + g * pinf) / (g - 1.0) + 0.5 * rho * (W[1] ** 2 + W[2] ** 2 + W[3] ** 2)
        U = [rho, rho * W[1], rho * W[2], rho * W[3], E]
        F = [rho * u, rho * u * W[1], rho * u * W[2], rho * u * W[3], u * (E + p)]
        F[1 + d] = F[1 + d] + p
        fac = (s - u) / (s - sstar)
        S = [fac * rho, fac * (rho * W[1]), fac * (rho * W[2]), fac * (rho * W[3]),
             fac * (E + (sstar - u) * (rho * sstar + p / (s - u)))]
        S[1 + d] = fac * (rho * sstar)
        return U, F, S

    UL_, FL, SL = state(WL, sL, uL)
    UR_, FR, SR = state(WR, sR, uR)
    sg = torch.sign(sstar)
    wl, wr = (1.0 + sg) / 2.0, (1.0 - sg) / 2.0
    return [wl * (FL[m] + sminus * (SL[m] - UL_[m])) + wr * (FR[m] + splus * (SR[m] - UR_[m])) for m in range(5)]


def rhs(cfg, U: torch.Tensor) -> torch.Tensor:
    """R(U) of Eq. (FVD) for the Euler equations; U: (5, nz, ny, nx) float64."""
    assert cfg.model == 0, "single-phase Euler only"
    eps = cfg.weno_eps if cfg.weno_eps > 0 else 1e-40
    Wp = cons_to_prim(cfg, pad(cfg, U))
    nz, ny, nx = cfg.nz, cfg.ny, cfg.nx
    R = torch.zeros_like(U)
    h = (cfg.dx, cfg.dy, cfg.dz)
    for d in range(3):
        n = (nx, ny, nz)[d]
        # interior in the two other axes, full halo along d; axis d moved last
        if d == 0:
            W = [w[H:H + nz, H:H + ny, :] for w in Wp]
        elif d == 1:
            W = [w[H:H + nz, :, H:H + nx].transpose(1, 2) for w in Wp]
        else:
            W = [w[:, H:H + ny, H:H + nx].permute(1, 2, 0) for w in Wp]
        # face f (0 .. n) lies between cells f-1 and f: padded positions f+2 | f+3
        sl = [lambda w, k=k: w[..., k:k + n + 1] for k in range(6)]
        WLf = [weno5z(sl[0](w), sl[1](w), sl[2](w), sl[3](w), sl[4](w), eps) for w in W]
        WRf = [weno5z(sl[5](w), sl[4](w), sl[3](w), sl[2](w), sl[1](w), eps) for w in W]
        F = hllc(cfg, d, WLf, WRf)
        dF = torch.stack([(f[..., 1:] - f[..., :-1]) / h[d] for f in F])
        if d == 1:
            dF = dF.transpose(2, 3)
        elif d == 2:
            dF = dF.permute(0, 3, 1, 2)
        R = R - dF
    return R


def rhs_vjp(cfg, U: torch.Tensor, Rbar: torch.Tensor) -> torch.Tensor:
    """(dR/dU)^T Rbar by one backward pass through rhs."""
    U = U.detach().clone().requires_grad_(True)
    R = rhs(cfg, U)
    (g,) = torch.autograd.grad(R, U, Rbar)
    return g


def rhs_jvp(cfg, U: torch.Tensor, V: torch.Tensor) -> torch.Tensor:
    """(dR/dU) V by forward-mode differentiation of rhs."""
    _, t = torch.func.jvp(lambda x: rhs(cfg, x), (U,), (V,))
    return t


def rk3_step(cfg, U: torch.Tensor, dt: float) -> torch.Tensor:
    """TVD-RK3 step in Shu-Osher form (Sec. 3.4)."""
    U1 = U + dt * rhs(cfg, U)
    U2 = 0.75 * U + 0.25 * U1 + 0.25 * dt * rhs(cfg, U1)
    return U / 3.0 + 2.0 / 3.0 * U2 + 2.0 / 3.0 * dt * rhs(cfg, U2)


def rk3_step_vjp(cfg, U: torch.Tensor, dt: float, Ubar: torch.Tensor) -> torch.Tensor:
    """Cotangent of U_n from the cotangent of U_{n+1} of one step (fixed dt)."""
    U = U.detach().clone().requires_grad_(True)
    (g,) = torch.autograd.grad(rk3_step(cfg, U, dt), U, Ubar)
    return g
