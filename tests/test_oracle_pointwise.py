"""Pins of the oracle's point-wise building blocks against what the mathematics
fixes: WENO5-Z (Sec. 3.2 step 3), HLLC (Sec. 3.2 step 6 + HLLC appendix) and the
stiffened-gas / mixture equation of state (Sec. 2.4)."""
import math

import numpy as np
import pytest

import oracle as O

RNG = np.random.default_rng(20240205)


# ---------------------------------------------------------------- WENO5-Z
def test_weno_constant_is_exact():
    for q in (1.0, -3.7, 71.42857142857143, 1e-8, 1e9):
        assert O.weno5z(q, q, q, q, q) == pytest.approx(q, rel=4e-16, abs=0)


def test_weno_reproduces_quadratic_cell_averages_exactly():
    # cell averages of any quadratic make every candidate interpolant exact, so the
    # face value is exact whatever the nonlinear weights are
    for _ in range(50):
        a0, a1, a2 = RNG.normal(size=3)
        h = 10 ** RNG.uniform(-3, 0)
        x0 = RNG.uniform(-1, 1)

        def avg(i):
            lo, hi = x0 + (i - 0.5) * h, x0 + (i + 0.5) * h
            prim = lambda x: a0 * x + a1 * x * x / 2 + a2 * x ** 3 / 3
            return (prim(hi) - prim(lo)) / h

        v = [avg(i) for i in range(-2, 3)]
        xf = x0 + 0.5 * h
        exact = a0 + a1 * xf + a2 * xf * xf
        scale = abs(a0) + abs(a1) + abs(a2)
        assert abs(O.weno5z(*v) - exact) < 1e-12 * scale
        # right-biased value at the same face uses the mirrored stencil
        w = [avg(i) for i in range(3, -2, -1)]
        assert abs(O.weno5z(*w) - exact) < 1e-12 * scale


def test_weno_linear_limit_is_fifth_order_upwind_interpolant():
    # eps -> huge makes alpha_k = d_k: the optimal linear scheme (2,-13,47,27,-3)/60
    for _ in range(50):
        v = RNG.normal(size=5)
        lin = (2 * v[0] - 13 * v[1] + 47 * v[2] + 27 * v[3] - 3 * v[4]) / 60.0
        assert O.weno5z(*v, eps=1e300) == pytest.approx(lin, rel=1e-14, abs=1e-15)


def test_weno_step_picks_smooth_stencil():
    # jump between cells i and i+1: the left-biased value comes from S0 = {0,0,0}
    assert abs(O.weno5z(0.0, 0.0, 0.0, 1.0, 1.0)) < 1e-12
    assert abs(O.weno5z(1.0, 1.0, 1.0, 0.0, 0.0) - 1.0) < 1e-12
    # a step one cell further left: value should stay within the data range
    val = O.weno5z(0.0, 0.0, 1.0, 1.0, 1.0)
    assert 0.0 <= val <= 1.0 + 1e-12


def test_weno_fifth_order_on_smooth_data():
    # face values from exact cell averages of exp(sin x); error ~ h^5 away from extrema
    errs = []
    for n in (40, 80, 160, 320):
        h = 2 * math.pi / n
        xs = np.arange(n) * h
        # exact averages by high-order Gauss quadrature
        gx, gw = np.polynomial.legendre.leggauss(8)
        f = lambda x: np.exp(np.sin(x))
        avg = np.array([(gw * f(x + h / 2 + gx * h / 2)).sum() / 2 for x in xs])
        e = 0.0
        for i in range(n):
            v = [avg[(i + k) % n] for k in (-2, -1, 0, 1, 2)]
            xf = xs[i] + h
            e = max(e, abs(O.weno5z(*v) - f(xf)))
        errs.append(e)
    slopes = [math.log2(errs[k] / errs[k + 1]) for k in range(3)]
    assert slopes[-1] > 4.5, slopes


# ---------------------------------------------------------------- states
def rand_state(model, rng=RNG):
    if model == O.DIM:
        a = rng.uniform(0.05, 0.95)
        return np.array([a * rng.uniform(0.5, 2), (1 - a) * rng.uniform(0.5, 2), *rng.normal(size=3),
                         rng.uniform(0.5, 3), a])
    return np.array([rng.uniform(0.3, 3), *rng.normal(size=3), rng.uniform(0.3, 3)])


def cfg_for(model, **kw):
    base = dict(nx=1, ny=1, nz=1, model=model)
    if model == O.DIM:
        base.update(gamma1=1.66, gamma2=1.4, pinf1=0.0, pinf2=0.5)
    base.update(kw)
    return O.Config(**base)


def physical_flux(model, d, W, g1=1.4, pinf1=0.0, g2=1.4, pinf2=0.0):
    """F^c of Eq. (convective_fluxes[_dim]) from its definition."""
    if model == O.DIM:
        a1 = W[6]
        inv = a1 / (g1 - 1) + (1 - a1) / (g2 - 1)
        gp = a1 * g1 * pinf1 / (g1 - 1) + (1 - a1) * g2 * pinf2 / (g2 - 1)
        rho = W[0] + W[1]
        vel = W[2:5]
        p = W[5]
        E = inv * p + gp + 0.5 * rho * vel @ vel
        un = vel[d]
        F = [W[0] * un, W[1] * un, *(rho * un * vel + p * np.eye(3)[d]), un * (E + p), a1 * un]
        return np.array(F)
    rho, vel, p = W[0], W[1:4], W[4]
    E = (p + g1 * pinf1) / (g1 - 1) + 0.5 * rho * vel @ vel
    un = vel[d]
    return np.array([rho * un, *(rho * un * vel + p * np.eye(3)[d]), un * (E + p)])


@pytest.mark.parametrize("model", [O.EULER, O.DIM])
def test_hllc_consistency(model):
    cfg = cfg_for(model)
    for _ in range(30):
        W = rand_state(model)
        for d in range(3):
            F, uh = O.hllc(cfg, d, W, W)
            ref = physical_flux(model, d, W, cfg.gamma1, cfg.pinf1, cfg.gamma2, cfg.pinf2)
            assert np.allclose(F, ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
            vel0 = 2 if model == O.DIM else 1
            assert uh == pytest.approx(W[vel0 + d], rel=1e-13, abs=1e-14)


@pytest.mark.parametrize("model", [O.EULER, O.DIM])
def test_hllc_supersonic_upwinding(model):
    cfg = cfg_for(model)
    vel0 = 2 if model == O.DIM else 1
    for _ in range(20):
        WL = rand_state(model)
        WR = rand_state(model)
        for d in range(3):
            L = WL.copy(); R = WR.copy()
            L[vel0 + d] = 8.0; R[vel0 + d] = 9.0     # everything moves right, faster than sound
            F, _ = O.hllc(cfg, d, L, R)
            assert np.array_equal(F, F)  # finite
            ref = physical_flux(model, d, L, cfg.gamma1, cfg.pinf1, cfg.gamma2, cfg.pinf2)
            assert np.allclose(F, ref, rtol=1e-14, atol=1e-14)
            L[vel0 + d] = -9.0; R[vel0 + d] = -8.0
            F, _ = O.hllc(cfg, d, L, R)
            ref = physical_flux(model, d, R, cfg.gamma1, cfg.pinf1, cfg.gamma2, cfg.pinf2)
            assert np.allclose(F, ref, rtol=1e-14, atol=1e-14)


def test_hllc_stationary_contact_is_exact():
    cfg = cfg_for(O.EULER)
    for _ in range(20):
        p = RNG.uniform(0.5, 2)
        WL = np.array([RNG.uniform(0.2, 5), 0.0, RNG.normal(), RNG.normal(), p])
        WR = np.array([RNG.uniform(0.2, 5), 0.0, RNG.normal(), RNG.normal(), p])
        F, uh = O.hllc(cfg, 0, WL, WR)
        assert F[0] == 0.0 and F[2] == 0.0 and F[3] == 0.0 and F[4] == 0.0
        assert F[1] == p
        assert uh == 0.0


def test_hllc_moving_contact_upwinds_density():
    cfg = cfg_for(O.EULER)
    for a in (0.3, -0.7):
        WL = np.array([2.0, a, 0.1, 0.0, 1.0])
        WR = np.array([0.5, a, -0.2, 0.0, 1.0])
        F, uh = O.hllc(cfg, 0, WL, WR)
        up = WL if a > 0 else WR
        assert F[0] == pytest.approx(up[0] * a, rel=1e-13)
        assert uh == pytest.approx(a, rel=1e-13)


@pytest.mark.parametrize("model", [O.EULER, O.DIM])
def test_hllc_mirror_antisymmetry_bitwise(model):
    cfg = cfg_for(model)
    vel0 = 2 if model == O.DIM else 1
    for _ in range(40):
        WL = rand_state(model)
        WR = rand_state(model)
        for d in range(3):
            F, uh = O.hllc(cfg, d, WL, WR)
            mL = WR.copy(); mR = WL.copy()
            mL[vel0 + d] *= -1; mR[vel0 + d] *= -1
            Fm, uhm = O.hllc(cfg, d, mL, mR)
            sign = np.ones_like(F)
            if model == O.DIM:
                sign[[0, 1, 2, 3, 4, 5, 6]] = -1
            else:
                sign[:] = -1
            sign[vel0 + d] = 1   # normal momentum flux is even under the mirror
            assert np.array_equal(Fm, sign * F), (d, Fm, F)
            assert uhm == -uh


# ---------------------------------------------------------------- EOS
@pytest.mark.parametrize("model", [O.EULER, O.NS, O.DIM])
def test_prim_cons_round_trip(model):
    cfg = O.Config(nx=4, ny=3, nz=2, model=model, gamma1=1.66 if model == O.DIM else 1.4,
                   gamma2=6.12, pinf2=3.43)
    W = np.stack([rand_state(O.DIM if model == O.DIM else O.EULER) for _ in range(24)], axis=1)
    W = W.reshape(cfg.shape)
    U = O.prim_to_cons(cfg, W)
    W2 = O.cons_to_prim(cfg, U)
    assert np.allclose(W2, W, rtol=1e-13, atol=1e-13)


def test_mixture_closure_limits():
    # alpha1 = 1 (0): the mixture is fluid 1 (2); E = (p + gamma pinf)/(gamma-1) + KE
    g1, p1, g2, p2 = 6.12, 3.43e8, 1.4, 0.0
    cfg = O.Config(nx=2, ny=1, nz=1, model=O.DIM, gamma1=g1, pinf1=p1, gamma2=g2, pinf2=p2)
    W = np.array([[1000.0, 0.0], [0.0, 1.2], [1.0, 3.0], [0.0, 0.0], [0.0, 0.0], [1e9, 1e5], [1.0, 0.0]])
    U = O.prim_to_cons(cfg, W.reshape(cfg.shape)).reshape(7, 2)
    E1 = (1e9 + g1 * p1) / (g1 - 1) + 0.5 * 1000.0 * 1.0
    E2 = (1e5 + g2 * p2) / (g2 - 1) + 0.5 * 1.2 * 9.0
    assert U[5, 0] == pytest.approx(E1, rel=1e-15)
    assert U[5, 1] == pytest.approx(E2, rel=1e-15)
