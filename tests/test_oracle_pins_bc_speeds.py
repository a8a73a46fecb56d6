"""Further pins of the oracle, CPU only.

* Symmetry boundaries (Sec. 3.1: the halo is the mirror image of the interior
  with the normal velocity negated): R on a box with a symmetry face equals,
  bit for bit, R on the box doubled across that face by explicit mirroring
  (mirrored cells with the normal momentum negated, zero-gradient outer ends),
  restricted to the original cells.  A halo mirrored about the wrong index, a
  velocity not negated, or a tangential one negated fails it.
* Einfeldt signal speeds (HLLC appendix, with the Roe-averaged u-bar and
  Einfeldt's c-bar of the reading): for data joined by one shock, Roe's
  linearisation reproduces the shock speed exactly, which fixes Einfeldt's
  s_R (and by mirroring s_L) in closed form from the Rankine-Hugoniot state and
  makes it bound the shock.  A c-bar without the velocity-jump term, with the
  Roe weight (gamma - 1)/2, or built from the arithmetic means fails it.  (The
  bound is not a theorem for colliding two-shock data: a light gas hit from
  both sides can have an exact shock faster than s_R.)
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2402_05193_amd import workloads as WL

MAT = {O.EULER: {}, O.NS: dict(mu=0.03, prandtl=0.7), O.DIM: dict(gamma1=1.66, gamma2=1.4)}


def doubled(W, axis, side, model):
    """W doubled across its low (side 0) or high (side 1) face along axis
    (0 = x): the mirror image with the normal velocity negated next to it."""
    ax = 3 - axis
    v = 2 if model == O.DIM else 1
    M = np.flip(W, axis=ax).copy()
    M[v + axis] *= -1.0
    return np.concatenate([M, W] if side == 0 else [W, M], axis=ax)


@pytest.mark.parametrize("model", [O.EULER, O.NS, O.DIM])
@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("side", [0, 1])
def test_symmetry_boundary_equals_mirrored_domain(model, axis, side):
    n = [9, 8, 7]
    case = WL.smooth_random(*n, model=model, seed=11 + axis, bc=(O.PERIODIC,) * 6, **MAT[model])
    bc = [O.ZERO_GRADIENT] * 6
    bc[2 * axis + side] = O.SYMMETRY
    kw = case.cfg_kwargs()
    kw.update(bc=tuple(bc))
    cfg = O.Config(**kw)
    U = O.prim_to_cons(cfg, case.W)
    R = O.rhs(cfg, U, dt=1e-5)
    W2 = doubled(case.W, axis, side, model)
    n2 = list(n)
    n2[axis] *= 2
    kw2 = dict(kw)
    kw2.update(nx=n2[0], ny=n2[1], nz=n2[2], bc=(O.ZERO_GRADIENT,) * 6)
    cfg2 = O.Config(**kw2)
    R2 = O.rhs(cfg2, O.prim_to_cons(cfg2, W2), dt=1e-5)
    sl = [slice(None)] * 4
    sl[3 - axis] = slice(n[axis], None) if side == 0 else slice(0, n[axis])
    assert np.array_equal(R, R2[tuple(sl)])


@pytest.mark.parametrize("gamma", [1.4, 1.67])
@pytest.mark.parametrize("mach", [1.05, 1.22, 2.0, 5.0, 20.0])
def test_einfeldt_speed_of_an_isolated_shock(gamma, mach):
    """Data joined by one shock of speed S (Rankine-Hugoniot, closed form): Roe's
    linearisation has u-bar + c-bar_Roe = S exactly (Roe 1981), with
    c-bar_Roe^2 = c-bar_E^2 - (1 - (gamma - 1)) / 2 * sqrt(rhoL rhoR) du^2 / (sqrtL + sqrtR)^2
    for an ideal gas (Einfeldt's c-bar has the weight 1/2 where the Roe average has
    (gamma - 1)/2).  So s_R = u-bar + sqrt((S - u-bar)^2 + (2 - gamma)/2 q^2) >= S,
    and the mirrored (left-facing) shock gives s_L = -s_R."""
    rho1, p1 = 1.3, 0.7
    rho2, u2, p2, S = WL.rankine_hugoniot(mach, gamma, rho1, p1)
    cfg = O.Config(nx=1, ny=1, nz=1, model=O.EULER, gamma1=gamma)
    WLs = np.array([rho2, u2, 0.0, 0.0, p2])
    WRs = np.array([rho1, 0.0, 0.0, 0.0, p1])
    sl, sr = O.hllc_speeds(cfg, 0, WLs, WRs)
    qL, qR = math.sqrt(rho2), math.sqrt(rho1)
    ubar = (qL * u2) / (qL + qR)
    q2 = qL * qR * u2 * u2 / (qL + qR) ** 2
    expect = ubar + math.sqrt((S - ubar) ** 2 + 0.5 * (2.0 - gamma) * q2)
    assert sr == pytest.approx(expect, rel=1e-13)
    assert sr >= S
    assert sl == pytest.approx(min(ubar - math.sqrt((S - ubar) ** 2 + 0.5 * (2.0 - gamma) * q2),
                                   u2 - math.sqrt(gamma * p2 / rho2)), rel=1e-13)
    # the mirrored shock moving left, along y
    ml = WRs.copy()
    mr = WLs.copy()
    mr[1] = 0.0
    mr[2] = -u2
    sl2, sr2 = O.hllc_speeds(cfg, 1, ml, mr)
    assert sl2 == pytest.approx(-sr, rel=1e-14)


def test_einfeldt_speeds_special_cases():
    cfg = O.Config(nx=1, ny=1, nz=1, model=O.EULER, gamma1=1.4)
    # equal states: u -/+ c
    W = np.array([1.3, 0.4, 0.0, 0.0, 2.0])
    c = math.sqrt(1.4 * 2.0 / 1.3)
    sl, sr = O.hllc_speeds(cfg, 0, W, W)
    assert sl == pytest.approx(0.4 - c, rel=1e-15)
    assert sr == pytest.approx(0.4 + c, rel=1e-15)
    # mirror: the speeds of the mirrored face are the negated, swapped ones
    WLs = np.array([2.0, 0.7, 0.1, 0.0, 5.0])
    WRs = np.array([0.3, -0.2, 0.0, 0.0, 0.4])
    sl, sr = O.hllc_speeds(cfg, 0, WLs, WRs)
    ml, mr = WRs.copy(), WLs.copy()
    ml[1] *= -1
    mr[1] *= -1
    sl2, sr2 = O.hllc_speeds(cfg, 0, ml, mr)
    assert sl2 == pytest.approx(-sr, rel=1e-15) and sr2 == pytest.approx(-sl, rel=1e-15)
