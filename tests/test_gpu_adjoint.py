"""Discrete adjoint on the GPU against the oracle's exact derivative.

The reference is oracle/euler_torch.py: the Euler right-hand side written with
plain torch operations (pinned to the C oracle and to central differences in
test_oracle_adjoint.py) differentiated by torch.autograd.  Bars (FP64): the
vector-Jacobian products of the right-hand side and of one TVD-RK3 step agree
to 1e-11 relative (max over the field); the dot-product identity
<J v, w> = <v, J^T w> holds to 1e-12; the gradient of a trajectory's kinetic
energy agrees with the oracle's to 1e-10 and with central finite differences
of the GPU forward solver within the accuracy finite differences allow.

WENO-Z epsilon: with eps = 1e-40 the derivative of the weights is singular at
constant stencils (zero-gradient halos, the uniform density and pressure of
the turbulence case): there the smoothness indicators are round-off (~1e-33)
and d/dbeta of tau/(beta + eps) is of order 1e50, so the result depends on the
rounding of each implementation.  Cases with constant stencils therefore use
eps = 1e-6 (the classical Jiang-Shu value); eps = 1e-40 is tested on fields in
general position (periodic and symmetry boundaries).
"""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import euler_torch as ET
from paper_2402_05193_amd import adjoint as AD
from paper_2402_05193_amd import solver as S
from paper_2402_05193_amd import workloads as WL

pytestmark = pytest.mark.gpu

MIXED = (WL.PERIODIC, WL.PERIODIC, WL.ZERO_GRADIENT, WL.ZERO_GRADIENT, WL.SYMMETRY, WL.SYMMETRY)


def rough(shape, bc, seed=1):
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    W = np.empty((5, nz, ny, nx))
    W[0] = 1 + 0.3 * rng.random((nz, ny, nx))
    W[1:4] = 0.3 * rng.standard_normal((3, nz, ny, nx))
    W[4] = 1 + 0.3 * rng.random((nz, ny, nx))
    return WL.Case(name="rough", nx=nx, ny=ny, nz=nz, dx=0.1, dy=0.12, dz=0.09, model=WL.EULER, bc=bc, W=W)


def turbulence_case(n, seed=0):
    h = 2 * np.pi / n
    return WL.Case(name="turbulence", nx=n, ny=n, nz=n, dx=h, dy=h, dz=h, model=WL.EULER, bc=(WL.PERIODIC,) * 6,
                   W=WL.decaying_turbulence(n, seed=seed))


EPS_SMOOTH = 1e-6  # WENO-Z epsilon of the cases with constant stencils

CASES = {  # name: (case, weno epsilon)
    "rough_periodic": (lambda: rough((13, 11, 9), (WL.PERIODIC,) * 6), 1e-40),
    "rough_symmetry": (lambda: rough((13, 11, 9), (WL.SYMMETRY,) * 6, seed=4), 1e-40),
    "rough_mixed_bc": (lambda: rough((12, 10, 8), MIXED, seed=2), EPS_SMOOTH),
    "rough_zero_gradient_line": (lambda: rough((24, 1, 1), (WL.ZERO_GRADIENT,) * 6, seed=3), EPS_SMOOTH),
    "smooth_mixed_bc": (lambda: WL.smooth_random(12, 10, 8, model=WL.EULER, seed=4, bc=MIXED), EPS_SMOOTH),
    "turbulence_16": (lambda: turbulence_case(16), EPS_SMOOTH),
}


def setup(case, eps=EPS_SMOOTH):
    oc = O.Config(**case.cfg_kwargs(), weno_eps=eps)
    U = O.prim_to_cons(oc, case.W)
    cfg = S.config_from_case(case, dtype=S.F64, weno_eps=eps)
    return oc, U, cfg


def setup_named(name):
    make, eps = CASES[name]
    return setup(make(), eps)


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel(a, b):
    return np.abs(a - b).max() / np.abs(b).max()


@pytest.mark.parametrize("name", list(CASES))
def test_rhs_adjoint_matches_oracle_vjp(name):
    oc, U, cfg = setup_named(name)
    rng = np.random.default_rng(5)
    Rbar = rng.standard_normal(U.shape)
    ref = ET.rhs_vjp(oc, torch.from_numpy(U), torch.from_numpy(Rbar)).numpy()
    Ubar = torch.empty_like(dev(U))
    S.rhs_adjoint(cfg, dev(U), dev(Rbar), Ubar)
    got = Ubar.cpu().numpy()
    r = rel(got, ref)
    print(f"{name}: rhs_adjoint rel {r:.3e}", flush=True)
    assert r <= 1e-11


def test_dot_product_identity():
    oc, U, cfg = setup_named("rough_periodic")
    rng = np.random.default_rng(6)
    v = rng.standard_normal(U.shape) * np.abs(U).max(axis=(1, 2, 3), keepdims=True)
    w = rng.standard_normal(U.shape)
    jv = ET.rhs_jvp(oc, torch.from_numpy(U), torch.from_numpy(v)).numpy()
    Ubar = torch.empty_like(dev(U))
    S.rhs_adjoint(cfg, dev(U), dev(w), Ubar)
    a = float((jv * w).sum())
    b = float((v * Ubar.cpu().numpy()).sum())
    assert abs(a - b) <= 1e-12 * abs(a)


@pytest.mark.parametrize("name", ["rough_periodic", "rough_mixed_bc", "turbulence_16"])
def test_rk3_step_adjoint_matches_oracle(name):
    oc, U, cfg = setup_named(name)
    dt = 0.3 * O.compute_dt(oc, U, 1.0)
    rng = np.random.default_rng(7)
    G = rng.standard_normal(U.shape)
    ref = ET.rk3_step_vjp(oc, torch.from_numpy(U), dt, torch.from_numpy(G)).numpy()
    Gd = dev(G)
    S.rk3_step_adjoint(cfg, dev(U), Gd, dt, S.adjoint_workspace(cfg))
    r = rel(Gd.cpu().numpy(), ref)
    print(f"{name}: rk3_step_adjoint rel {r:.3e}", flush=True)
    assert r <= 1e-11


@pytest.mark.parametrize("name", ["rough_periodic", "rough_mixed_bc", "turbulence_16"])
def test_rk3_step_adjoint_stages_matches_recomputing_sweep(name):
    """The sweep from given stage states (rk3_stage's U^(1), U^(2)) against the one
    that recomputes them, and against the oracle's VJP: the same up to the order of
    the atomic additions."""
    oc, U, cfg = setup_named(name)
    dt = 0.3 * O.compute_dt(oc, U, 1.0)
    rng = np.random.default_rng(11)
    G = rng.standard_normal(U.shape)
    ref = ET.rk3_step_vjp(oc, torch.from_numpy(U), dt, torch.from_numpy(G)).numpy()
    Ud = dev(U)
    U1 = torch.empty_like(Ud)
    U2 = torch.empty_like(Ud)
    S.rk3_stage(cfg, 1, Ud, Ud, U1, dt)
    S.rk3_stage(cfg, 2, Ud, U1, U2, dt)
    aws = S.adjoint_workspace(cfg)
    Ga = dev(G)
    Gb = dev(G)
    S.rk3_step_adjoint(cfg, Ud, Ga, dt, aws)
    S.rk3_step_adjoint_stages(cfg, Ud, U1, U2, Gb, dt, aws)
    a, b = Ga.cpu().numpy(), Gb.cpu().numpy()
    r_ab, r_ref = rel(b, a), rel(b, ref)
    print(f"{name}: rk3_step_adjoint_stages rel to recomputing sweep {r_ab:.3e}, to oracle {r_ref:.3e}", flush=True)
    assert r_ab <= 1e-13
    assert r_ref <= 1e-11


def test_trajectory_gradient_matches_oracle_and_checkpointing():
    """d KE(U_N) / d U_0 over N = 7 fixed-dt steps (checkpoint segments 3, 3, 1)
    against torch.autograd through the oracle's steps; the checkpoint spacing
    does not change the gradient beyond round-off."""
    oc, U, cfg = setup(turbulence_case(16, seed=3))
    dt = 0.5 * O.compute_dt(oc, U, 1.0)
    N = 7
    Ut = torch.from_numpy(U).requires_grad_(True)
    X = Ut
    for _ in range(N):
        X = ET.rk3_step(oc, X, dt)
    h3 = oc.dx * oc.dy * oc.dz
    loss = 0.5 * ((X[1] ** 2 + X[2] ** 2 + X[3] ** 2) / X[0]).sum() * h3
    (ref,) = torch.autograd.grad(loss, Ut)
    ref = ref.numpy()
    grads = []
    for every in (3, 1, N):
        U0 = dev(U).requires_grad_(True)
        L = AD.kinetic_energy(cfg, AD.advance_fixed_dt(cfg, U0, N, dt, every=every))
        (g,) = torch.autograd.grad(L, U0)
        grads.append(g.cpu().numpy())
        assert abs(float(L) - float(loss)) <= 1e-12 * abs(float(loss))
    r = rel(grads[0], ref)
    print(f"trajectory gradient rel {r:.3e}", flush=True)
    assert r <= 1e-10
    for g in grads[1:]:
        assert rel(g, grads[0]) <= 1e-13


def test_decaying_turbulence_gradient_vs_central_differences():
    """The differentiation workload: 64^3 decaying turbulence, kinetic energy
    after 100 fixed-dt steps, checkpoints every 10 steps; the gradient projected
    on 16 seeded directions against central differences of the forward solver.
    The discrete solver is only piecewise smooth: the min/max of the wave
    speeds, |beta0 - beta2| and the HLLC switch have kinks, and in a smooth
    field the candidates of each min/max nearly tie at every face, so over 100
    steps a perturbation of relative size 1e-4 .. 1e-6 crosses many kinks and
    central differences stall at 1e-2 .. 1e-4 (measured).  The exact derivative
    itself is checked against the oracle (previous test); here the bar is the
    best h of a short sweep: median over the 16 directions <= 1e-3, worst
    <= 5e-2."""
    n, N = 64, 100
    case = turbulence_case(n, seed=0)
    oc, U, cfg = setup(case)
    Ud = dev(U)
    dtd = torch.zeros(1, dtype=torch.float64, device="cuda")
    S.compute_dt(S.Config(**{**cfg.__dict__, "cfl": 0.5}), Ud, dtd, S.workspace(cfg))
    dt = float(dtd)
    U0 = Ud.clone().requires_grad_(True)
    L = AD.kinetic_energy(cfg, AD.advance_fixed_dt(cfg, U0, N, dt, every=10))
    (g,) = torch.autograd.grad(L, U0)
    ws = S.workspace(cfg)
    scale = torch.from_numpy(np.abs(U).max(axis=(1, 2, 3), keepdims=True)).cuda()

    def loss_at(X):
        X = X.clone()
        S.advance(cfg, X, N, dt, ws)
        return float(AD.kinetic_energy(cfg, X))

    errs, best = [], []
    for k in range(16):
        gen = torch.Generator(device="cpu").manual_seed(1000 + k)
        v = torch.randn(U.shape, generator=gen, dtype=torch.float64).cuda() * scale
        exact = float((g * v).sum())
        e = {}
        for h in (1e-4, 1e-6, 1e-8):
            fd = (loss_at(Ud + h * v) - loss_at(Ud - h * v)) / (2 * h)
            e[h] = abs(fd - exact) / abs(exact)
        errs.append(e[1e-6])
        best.append(min(e.values()))
        print(f"direction {k}: <g,v> {exact:.6e}  FD rel err h=1e-4 {e[1e-4]:.2e}  1e-6 {e[1e-6]:.2e}"
              f"  1e-8 {e[1e-8]:.2e}", flush=True)
    assert np.median(best) <= 1e-3
    assert max(best) <= 5e-2
