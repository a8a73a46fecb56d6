"""Exact solution of the one-dimensional Riemann problem for two stiffened gases.

Textbook construction (Toro, "Riemann Solvers and Numerical Methods for Fluid
Dynamics", ch. 4): the star pressure is the root of
f_L(p) + f_R(p) + (u_R - u_L) = 0, where each f_K is the shock (Rankine-
Hugoniot) or rarefaction (isentrope) relation of side K.  A stiffened gas
behaves like an ideal gas in the shifted pressure p + p_inf, so each side uses
its own (gamma_K, p_inf_K).  The contact separates the two materials.

This is an independent pin of the shock-tube results; it shares nothing with
the oracle or the HIP path.
"""
from __future__ import annotations

import math

import numpy as np


class Side:
    def __init__(self, rho, u, p, gamma, pinf=0.0):
        self.rho, self.u, self.p, self.g, self.pinf = rho, u, p, gamma, pinf
        self.c = math.sqrt(gamma * (p + pinf) / rho)

    def f(self, p):
        """Velocity jump across the K-wave as a function of the star pressure, and its derivative."""
        g, pk, pinf, rho, c = self.g, self.p, self.pinf, self.rho, self.c
        if p > pk:  # shock
            A = 2.0 / ((g + 1.0) * rho)
            B = (g - 1.0) / (g + 1.0) * (pk + pinf)
            q = math.sqrt(A / (p + pinf + B))
            return (p - pk) * q, q * (1.0 - 0.5 * (p - pk) / (p + pinf + B))
        r = (p + pinf) / (pk + pinf)
        e = (g - 1.0) / (2.0 * g)
        return 2.0 * c / (g - 1.0) * (r ** e - 1.0), 1.0 / (rho * c) * r ** (-(g + 1.0) / (2.0 * g))

    def rho_star(self, p):
        g, pk, pinf, rho = self.g, self.p, self.pinf, self.rho
        pb, pkb = p + pinf, pk + pinf
        if p > pk:
            r = pb / pkb
            gg = (g - 1.0) / (g + 1.0)
            return rho * (r + gg) / (gg * r + 1.0)
        return rho * (pb / pkb) ** (1.0 / g)


def star_state(L: Side, R: Side, tol: float = 1e-15):
    """Newton iteration for p* with a bisection safeguard; returns (p*, u*, residual)."""
    du = R.u - L.u
    lo = max(-L.pinf, -R.pinf) + 1e-300

    def F(p):
        fl, dl = L.f(p)
        fr, dr = R.f(p)
        return fl + fr + du, dl + dr

    # positivity of the star state for the given data (no vacuum)
    p = max(0.5 * (L.p + R.p), lo * 0.5 + 1e-12)
    a, b = lo, max(L.p, R.p) * 10.0 + 10.0
    while F(b)[0] < 0:
        b *= 10.0
    for _ in range(200):
        val, der = F(p)
        if val > 0:
            b = min(b, p)
        else:
            a = max(a, p)
        pn = p - val / der
        if not (a < pn < b):
            pn = 0.5 * (a + b)
        if abs(pn - p) <= tol * max(abs(pn), 1.0):
            p = pn
            break
        p = pn
    fl, _ = L.f(p)
    fr, _ = R.f(p)
    u = 0.5 * (L.u + R.u) + 0.5 * (fr - fl)
    return p, u, F(p)[0]


def sample(L: Side, R: Side, xi: np.ndarray):
    """(rho, u, p, material) at similarity coordinates xi = (x - x0) / t; material 0 = left fluid."""
    ps, us, _ = star_state(L, R)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    mat = np.empty(xi.shape, dtype=np.int8)
    for n, s in enumerate(xi):
        if s <= us:
            K, sign = L, -1.0
            mat[n] = 0
        else:
            K, sign = R, 1.0
            mat[n] = 1
        g, pinf, c = K.g, K.pinf, K.c
        if ps > K.p:  # shock on side K
            q = math.sqrt((g + 1.0) / (2.0 * g) * (ps + pinf) / (K.p + pinf) + (g - 1.0) / (2.0 * g))
            S = K.u + sign * c * q
            if (sign < 0 and s <= S) or (sign > 0 and s >= S):
                rho[n], u[n], p[n] = K.rho, K.u, K.p
            else:
                rho[n], u[n], p[n] = K.rho_star(ps), us, ps
        else:  # rarefaction on side K
            cs = c * ((ps + pinf) / (K.p + pinf)) ** ((g - 1.0) / (2.0 * g))
            head = K.u + sign * c
            tail = us + sign * cs
            outside = (s <= head) if sign < 0 else (s >= head)
            inside_star = (s >= tail) if sign < 0 else (s <= tail)
            if outside:
                rho[n], u[n], p[n] = K.rho, K.u, K.p
            elif inside_star:
                rho[n], u[n], p[n] = K.rho_star(ps), us, ps
            else:
                # fan: u - sign c = xi, Riemann invariant u + (-sign) 2c/(g-1) = const
                un = 2.0 / (g + 1.0) * (-sign * c + (g - 1.0) / 2.0 * K.u + s)
                cn = -sign * (un - s)
                rr = (cn / c) ** (2.0 / (g - 1.0))
                rho[n] = K.rho * rr
                u[n] = un
                p[n] = (K.p + pinf) * rr ** g - pinf
    return rho, u, p, mat
