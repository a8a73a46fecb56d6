"""Sixth-order central viscous fluxes (visc_order = 6; the paper's single-phase
setup) on the GPU against the oracle, through the C ABI (rhs_ws, rk3_step,
advance).  Bars as for the 4th-order fluxes: per component 1e-12 relative for
one RHS (or twice the case's round-off floor), 1e-10 for RK3 increments."""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2402_05193_amd import solver as S
from paper_2402_05193_amd import workloads as WL
from test_gpu_parity import RHS_TOL, comp_rel, dev, host, oracle_cfg, roundoff_floor, solver_cfg

pytestmark = pytest.mark.gpu

MIXED_BC = (WL.PERIODIC, WL.PERIODIC, WL.ZERO_GRADIENT, WL.ZERO_GRADIENT, WL.SYMMETRY, WL.SYMMETRY)
LAWS = {"const": {}, "sutherland": dict(visc_law=2, T_ref=0.8, sutherland=0.35, gas_R=0.7),
        "power": dict(visc_law=1, T_ref=0.9, gas_R=1.3)}


def cases():
    return {
        "ns_tgv24": WL.taylor_green(24, viscous=True, ma=0.3),
        "ns_ragged": WL.smooth_random(19, 13, 10, model=WL.NS, seed=22, bc=MIXED_BC, mu=0.02, prandtl=0.7),
        "ns_thin": WL.smooth_random(21, 3, 5, model=WL.NS, seed=31, bc=MIXED_BC, mu=0.05, prandtl=0.72),
        # several marched chunks along y (32 + 13) and z (32 + 32 + 6)
        "ns_chunks": WL.smooth_random(10, 45, 70, model=WL.NS, seed=37, bc=MIXED_BC, mu=0.03, prandtl=0.72),
        # one cell along an axis: that axis' stencils see the same cell (derivatives vanish)
        "ns_flat_y": WL.smooth_random(12, 1, 9, model=WL.NS, seed=41, bc=MIXED_BC, mu=0.04, prandtl=0.72),
        "ns_line_z": WL.smooth_random(1, 1, 40, model=WL.NS, seed=43, bc=MIXED_BC, mu=0.04, prandtl=0.72),
    }


@pytest.mark.parametrize("law", list(LAWS))
@pytest.mark.parametrize("name", list(cases()))
def test_rhs_parity_visc6(name, law):
    case = cases()[name]
    oc = oracle_cfg(case, visc_order=6, **LAWS[law])
    U = O.prim_to_cons(oc, case.W)
    print(f"[visc6] rhs {name} {law} shape={U.shape}", flush=True)
    Ro = O.rhs(oc, U)
    sc = solver_cfg(case, visc_order=6, **LAWS[law])
    Rd = torch.empty_like(dev(U))
    S.rhs(sc, dev(U), Rd, ws=S.workspace(sc))
    err = comp_rel(host(Rd), Ro)
    floor = roundoff_floor(oc, U, 0.0)
    print(f"[visc6] rhs {name} {law} rel err {np.array2string(err, precision=2)} "
          f"floor {np.array2string(floor, precision=2)}", flush=True)
    assert np.all(err <= np.maximum(RHS_TOL, 2.0 * floor)), (err, floor)
    # sixth order differs from fourth order
    R4 = O.rhs(oracle_cfg(case, **LAWS[law]), U)
    assert np.abs(Ro - R4).max() > 1e-9 * np.abs(R4).max()


@pytest.mark.parametrize("name", ["ns_ragged", "ns_tgv24"])
def test_rk3_step_parity_visc6(name):
    case = cases()[name]
    oc = oracle_cfg(case, visc_order=6)
    U = O.prim_to_cons(oc, case.W)
    dt = 0.4 * O.compute_dt(oc, U, 1.0)
    Uo = O.rk3_step(oc, U, dt)
    sc = solver_cfg(case, visc_order=6)
    Ud = dev(U)
    S.rk3_step(sc, Ud, dt, S.workspace(sc))
    err = comp_rel(host(Ud) - U, Uo - U)
    print(f"[visc6] rk3 step {name} increment rel err {np.array2string(err, precision=2)}", flush=True)
    assert np.all(err <= 1e-10), err


def test_single_phase_setup_advance():
    """The paper's single-phase setup: TENO6-A, 6th-order viscous fluxes, TVD-RK3
    at CFL 0.9; ten CFL-mode steps of the viscous Taylor-Green vortex at 24^3."""
    case = WL.taylor_green(24, viscous=True, ma=0.3)
    oc = oracle_cfg(case, visc_order=6, scheme=1)
    U = O.prim_to_cons(oc, case.W)
    Uo, to = O.advance(oc, U, 10, 0.0, cfl=0.9)
    sc = solver_cfg(case, visc_order=6, scheme=1, cfl=0.9)
    Ud = dev(U)
    t = S.advance(sc, Ud, 10, 0.0, S.workspace(sc), t=0.0)
    assert abs(t - to) <= 1e-12 * to
    err = comp_rel(host(Ud), Uo)
    # the trajectory's own round-off floor (oracle rerun from U moved by an ulp)
    rng = np.random.default_rng(3)
    Up = U * (1.0 + rng.choice([-1.0, 1.0], size=U.shape) * 2.0 ** -53)
    Uop, _ = O.advance(oc, Up, 10, 0.0, cfl=0.9)
    floor = comp_rel(Uop, Uo)
    print(f"[visc6] single-phase setup advance rel err {np.array2string(err, precision=2)} "
          f"floor {np.array2string(floor, precision=2)}", flush=True)
    assert np.all(err <= np.maximum(1e-12, 4.0 * floor)), (err, floor)


def test_rhs_without_workspace_is_refused():
    case = cases()["ns_tgv24"]
    sc = solver_cfg(case, visc_order=6)
    U = dev(O.prim_to_cons(oracle_cfg(case), case.W))
    R = torch.empty_like(U)
    c = sc.c_struct()
    import ctypes
    assert S.lib().rhs(ctypes.byref(c), S._ptr(U), S._ptr(R), 0.0, None) == S.EUNSUPPORTED


def test_fp32_visc6_error_statement():
    case = cases()["ns_ragged"]
    oc = oracle_cfg(case, visc_order=6, **LAWS["sutherland"])
    U = O.prim_to_cons(oc, case.W)
    Ro = O.rhs(oc, U)
    sc = solver_cfg(case, dtype=S.F32, visc_order=6, **LAWS["sutherland"])
    Ud = dev(U, torch.float32)
    Rd = torch.empty_like(Ud)
    S.rhs(sc, Ud, Rd, ws=S.workspace(sc))
    err = comp_rel(host(Rd), Ro)
    print(f"[visc6] FP32 rel err {np.array2string(err, precision=2)}", flush=True)
    assert np.all(err <= 1e-3), err
