"""Temperature-dependent viscosity (Sec. 2.5: power law, Sutherland's law) on
the GPU against the oracle, through the C ABI.  Bars as for constant
viscosity: 1e-12 per component for one RHS (or twice the case's round-off
floor), 1e-10 after several CFL-mode steps, the CFL time step to 1e-13."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2402_05193_amd import solver as S
from paper_2402_05193_amd import workloads as WL
from test_gpu_parity import RHS_TOL, comp_rel, dev, host, oracle_cfg, roundoff_floor, solver_cfg

pytestmark = pytest.mark.gpu

MIXED_BC = (WL.PERIODIC, WL.PERIODIC, WL.ZERO_GRADIENT, WL.ZERO_GRADIENT, WL.SYMMETRY, WL.SYMMETRY)

LAWS = {
    "power": dict(visc_law=1, T_ref=0.9, sutherland=0.0, gas_R=1.3),
    "sutherland": dict(visc_law=2, T_ref=0.8, sutherland=0.35, gas_R=0.7),
}


def law_cases():
    return {
        "ns_tgv24": WL.taylor_green(24, viscous=True, ma=0.3),
        "ns_ragged": WL.smooth_random(19, 13, 10, model=WL.NS, seed=22, bc=MIXED_BC, mu=0.02, prandtl=0.7),
    }


@pytest.mark.parametrize("law", list(LAWS))
@pytest.mark.parametrize("name", list(law_cases()))
def test_rhs_parity_viscosity_law(name, law):
    case = law_cases()[name]
    oc = oracle_cfg(case, **LAWS[law])
    U = O.prim_to_cons(oc, case.W)
    Ro = O.rhs(oc, U)
    sc = solver_cfg(case, **LAWS[law])
    Rd = torch.empty_like(dev(U))
    S.rhs(sc, dev(U), Rd)
    err = comp_rel(host(Rd), Ro)
    floor = roundoff_floor(oc, U, 0.0)
    print(f"[visc] {name} {law} rel err {np.array2string(err, precision=2)} "
          f"floor {np.array2string(floor, precision=2)}", flush=True)
    assert np.all(err <= np.maximum(RHS_TOL, 2.0 * floor)), (err, floor)
    # the law changes the result (it is not silently constant)
    R0 = O.rhs(oracle_cfg(case), U)
    assert np.abs(Ro - R0).max() > 1e-6 * np.abs(R0).max()


@pytest.mark.parametrize("law", list(LAWS))
def test_cfl_and_advance_with_viscosity_law(law):
    case = WL.smooth_random(16, 12, 10, model=WL.NS, seed=9, mu=0.4, prandtl=0.72)
    oc = oracle_cfg(case, **LAWS[law])
    U = O.prim_to_cons(oc, case.W)
    sc = solver_cfg(case, cfl=0.5, **LAWS[law])
    dt_o = O.compute_dt(oc, U, 0.5)
    dtd = torch.zeros(1, dtype=torch.float64, device="cuda")
    S.compute_dt(sc, dev(U), dtd, S.workspace(sc))
    assert abs(float(dtd) - dt_o) <= 1e-13 * dt_o
    Uo, to = O.advance(oc, U, 5, 0.0, cfl=0.5)
    Ud = dev(U)
    t = S.advance(sc, Ud, 5, 0.0, S.workspace(sc), t=0.0)
    assert abs(t - to) <= 1e-12 * to
    err = comp_rel(host(Ud) - U, Uo - U)
    print(f"[visc] advance {law} increment rel err {np.array2string(err, precision=2)}", flush=True)
    assert np.all(err <= 1e-10), err


def test_fp32_viscosity_law_error_statement():
    case = law_cases()["ns_ragged"]
    oc = oracle_cfg(case, **LAWS["sutherland"])
    U = O.prim_to_cons(oc, case.W)
    Ro = O.rhs(oc, U)
    sc = solver_cfg(case, dtype=S.F32, **LAWS["sutherland"])
    Ud = dev(U, torch.float32)
    Rd = torch.empty_like(Ud)
    S.rhs(sc, Ud, Rd)
    err = comp_rel(host(Rd), Ro)
    print(f"[visc] FP32 sutherland rel err {np.array2string(err, precision=2)}", flush=True)
    assert np.all(err <= 1e-3), err
