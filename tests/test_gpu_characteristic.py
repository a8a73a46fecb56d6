"""Characteristic-variable reconstruction (recon = 1) on the GPU against the
oracle's (Sec. 3.2 steps 1-4), through the C ABI.  Same bars as the primitive
reconstruction: per component 1e-12 relative for one RHS, or twice the case's
measured round-off floor where that is larger."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2402_05193_amd import solver as S
from paper_2402_05193_amd import workloads as WL
from test_gpu_parity import RHS_TOL, cases, comp_rel, dev, host, oracle_cfg, roundoff_floor, solver_cfg

pytestmark = pytest.mark.gpu

NAMES = ["euler_tgv32", "euler_ragged", "euler_line", "euler_plane", "ns_tgv32", "ns_ragged", "dim_smooth",
         "dim_ragged", "dim_sbi"]


@pytest.fixture(scope="module")
def all_cases():
    return cases()


@pytest.mark.parametrize("name", NAMES)
def test_rhs_parity_characteristic(all_cases, name):
    case = all_cases[name]
    oc = oracle_cfg(case, recon=1)
    U = O.prim_to_cons(oc, case.W)
    dt = 0.3 * O.compute_dt(oc, U, 1.0)
    print(f"[char] rhs {name} shape={U.shape}", flush=True)
    Ro = O.rhs(oc, U, dt=dt)
    sc = solver_cfg(case, recon=1)
    Ud = dev(U)
    Rd = torch.empty_like(Ud)
    S.rhs(sc, Ud, Rd, dt=dt)
    err = comp_rel(host(Rd), Ro)
    floor = roundoff_floor(oc, U, dt)
    tol = np.maximum(RHS_TOL, 2.0 * floor)
    print(f"[char] rhs {name} rel err {np.array2string(err, precision=2)} "
          f"floor {np.array2string(floor, precision=2)}", flush=True)
    assert np.all(err <= tol), (err, floor)


@pytest.mark.parametrize("name", ["euler_ragged", "dim_sbi", "ns_ragged"])
def test_rk3_step_parity_characteristic(all_cases, name):
    case = all_cases[name]
    oc = oracle_cfg(case, recon=1)
    U = O.prim_to_cons(oc, case.W)
    dt = 0.4 * O.compute_dt(oc, U, 1.0)
    Uo = O.rk3_step(oc, U, dt)
    sc = solver_cfg(case, recon=1)
    Ud = dev(U)
    S.rk3_step(sc, Ud, dt, S.workspace(sc))
    err = comp_rel(host(Ud) - U, Uo - U)   # the increment, relative to its own size
    print(f"[char] rk3 step {name} increment rel err {np.array2string(err, precision=2)}", flush=True)
    assert np.all(err <= 1e-10), err


def test_uniform_state_and_conservation_characteristic():
    for model, state in ((WL.EULER, (1.0, 0.1, -0.2, 0.3, 1.0)), (WL.DIM, (0.3, 0.5, 0.2, -0.1, 0.4, 1.3, 0.4))):
        case = WL.uniform(9, 8, 7, model=model, state=state, gamma2=1.66)
        sc = solver_cfg(case, recon=1)
        U = O.prim_to_cons(oracle_cfg(case), case.W)
        Rd = torch.empty_like(dev(U))
        S.rhs(sc, dev(U), Rd)
        assert bool((Rd == 0).all())
    case = WL.smooth_random(16, 12, 10, model=WL.EULER, seed=5)
    sc = solver_cfg(case, recon=1)
    U = O.prim_to_cons(oracle_cfg(case), case.W)
    Rd = torch.empty_like(dev(U))
    S.rhs(sc, dev(U), Rd)
    R = host(Rd)
    for m in range(5):
        assert abs(R[m].sum()) <= 1e-13 * np.abs(R[m]).sum()


def test_fp32_characteristic_error_statement(all_cases):
    """FP32 characteristic reconstruction against the FP64 oracle (stated)."""
    for name in ("euler_ragged", "dim_smooth"):
        case = all_cases[name]
        oc = oracle_cfg(case, recon=1)
        U = O.prim_to_cons(oc, case.W)
        Ro = O.rhs(oc, U)
        sc = solver_cfg(case, dtype=S.F32, recon=1)
        Ud = dev(U, torch.float32)
        Rd = torch.empty_like(Ud)
        S.rhs(sc, Ud, Rd)
        err = comp_rel(host(Rd), Ro)
        print(f"[char] FP32 {name} rel err {np.array2string(err, precision=2)}", flush=True)
        assert np.all(err <= 5e-3), err
