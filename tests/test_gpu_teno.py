"""TENO6-A reconstruction (scheme = 1; Sec. 3.2 step 3) on the GPU against the
oracle, through the C ABI, for primitive (recon = 0) and characteristic
(recon = 1) variables.  Bars as for WENO5-Z: per component 1e-12 relative for
one RHS, or twice the case's measured round-off floor where that is larger;
RK3 increments 1e-10.  The cases with discontinuities (shock tube, shock-bubble)
exercise the stencil cut-off: there the two sides must drop the same stencils."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2402_05193_amd import solver as S
from paper_2402_05193_amd import workloads as WL
from test_gpu_parity import RHS_TOL, cases, comp_rel, dev, host, oracle_cfg, roundoff_floor, solver_cfg

pytestmark = pytest.mark.gpu

NAMES = ["euler_tgv32", "euler_ragged", "euler_line", "euler_plane", "ns_tgv32", "ns_ragged", "dim_smooth",
         "dim_ragged", "dim_sbi", "euler_sod"]


@pytest.fixture(scope="module")
def all_cases():
    c = cases()
    c["euler_sod"] = WL.sod_tube(96)
    return c


@pytest.mark.parametrize("recon", [0, 1])
@pytest.mark.parametrize("name", NAMES)
def test_rhs_parity_teno(all_cases, name, recon):
    case = all_cases[name]
    oc = oracle_cfg(case, scheme=1, recon=recon)
    U = O.prim_to_cons(oc, case.W)
    dt = 0.3 * O.compute_dt(oc, U, 1.0)
    print(f"[teno] rhs {name} recon={recon} shape={U.shape}", flush=True)
    Ro = O.rhs(oc, U, dt=dt)
    sc = solver_cfg(case, scheme=1, recon=recon)
    Ud = dev(U)
    Rd = torch.empty_like(Ud)
    S.rhs(sc, Ud, Rd, dt=dt)
    err = comp_rel(host(Rd), Ro)
    floor = roundoff_floor(oc, U, dt)
    tol = np.maximum(RHS_TOL, 2.0 * floor)
    print(f"[teno] rhs {name} recon={recon} rel err {np.array2string(err, precision=2)} "
          f"floor {np.array2string(floor, precision=2)}", flush=True)
    assert np.all(err <= tol), (err, floor)


@pytest.mark.parametrize("recon", [0, 1])
@pytest.mark.parametrize("name", ["euler_ragged", "dim_sbi", "ns_ragged", "euler_sod"])
def test_rk3_step_parity_teno(all_cases, name, recon):
    case = all_cases[name]
    oc = oracle_cfg(case, scheme=1, recon=recon)
    U = O.prim_to_cons(oc, case.W)
    dt = 0.4 * O.compute_dt(oc, U, 1.0)
    Uo = O.rk3_step(oc, U, dt)
    sc = solver_cfg(case, scheme=1, recon=recon)
    Ud = dev(U)
    S.rk3_step(sc, Ud, dt, S.workspace(sc))
    err = comp_rel(host(Ud) - U, Uo - U)
    print(f"[teno] rk3 step {name} recon={recon} increment rel err {np.array2string(err, precision=2)}",
          flush=True)
    assert np.all(err <= 1e-10), err


def test_advance_cfl_teno_tgv():
    """Twenty CFL-mode steps of the viscous Taylor-Green vortex at 32^3 with
    TENO6-A at CFL 0.9."""
    case = WL.taylor_green(32, viscous=True)
    oc = oracle_cfg(case, scheme=1)
    U = O.prim_to_cons(oc, case.W)
    Uo, to = O.advance(oc, U, 20, 0.0, cfl=0.9)
    sc = solver_cfg(case, scheme=1, cfl=0.9)
    Ud = dev(U)
    t = S.advance(sc, Ud, 20, 0.0, S.workspace(sc), t=0.0)
    assert abs(t - to) <= 1e-12 * to
    err = comp_rel(host(Ud), Uo)
    # the trajectory's own round-off floor: the oracle rerun from U moved by one
    # unit in the last place (the central six-point scheme damps no rounding)
    rng = np.random.default_rng(3)
    Up = U * (1.0 + rng.choice([-1.0, 1.0], size=U.shape) * 2.0 ** -53)
    Uop, _ = O.advance(oc, Up, 20, 0.0, cfl=0.9)
    floor = comp_rel(Uop, Uo)
    print(f"[teno] advance tgv32 rel err {np.array2string(err, precision=2)} "
          f"floor {np.array2string(floor, precision=2)}", flush=True)
    assert np.all(err <= np.maximum(1e-12, 4.0 * floor)), (err, floor)


def test_uniform_state_and_conservation_teno():
    for model, state in ((WL.EULER, (1.0, 0.1, -0.2, 0.3, 1.0)), (WL.DIM, (0.3, 0.5, 0.2, -0.1, 0.4, 1.3, 0.4))):
        case = WL.uniform(9, 8, 7, model=model, state=state, gamma2=1.66)
        for recon in (0, 1):
            sc = solver_cfg(case, scheme=1, recon=recon)
            U = O.prim_to_cons(oracle_cfg(case), case.W)
            Rd = torch.empty_like(dev(U))
            S.rhs(sc, dev(U), Rd)
            assert bool((Rd == 0).all())
    case = WL.smooth_random(16, 12, 10, model=WL.EULER, seed=5)
    sc = solver_cfg(case, scheme=1)
    U = O.prim_to_cons(oracle_cfg(case), case.W)
    Rd = torch.empty_like(dev(U))
    S.rhs(sc, dev(U), Rd)
    R = host(Rd)
    for m in range(5):
        assert abs(R[m].sum()) <= 1e-13 * np.abs(R[m]).sum()


def test_fp32_teno_error_statement(all_cases):
    """FP32 TENO6-A against the FP64 oracle (stated)."""
    for name, recon in (("euler_ragged", 0), ("dim_smooth", 1), ("ns_tgv32", 0)):
        case = all_cases[name]
        oc = oracle_cfg(case, scheme=1, recon=recon)
        U = O.prim_to_cons(oc, case.W)
        Ro = O.rhs(oc, U)
        sc = solver_cfg(case, dtype=S.F32, scheme=1, recon=recon)
        Ud = dev(U, torch.float32)
        Rd = torch.empty_like(Ud)
        S.rhs(sc, Ud, Rd)
        err = comp_rel(host(Rd), Ro)
        print(f"[teno] FP32 {name} recon={recon} rel err {np.array2string(err, precision=2)}", flush=True)
        assert np.all(err <= 5e-3), err
