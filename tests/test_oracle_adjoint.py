"""Pins of the adjoint's reference (oracle/euler_torch.py), CPU only.

The reference is a plain PyTorch FP64 implementation of the Euler right-hand
side whose derivative torch.autograd takes.  It is pinned to things other than
itself: its forward values equal the C oracle's right-hand side (which the
accuracy and invariant tests pin to the paper), and its derivative equals
central finite differences of the forward operator with the O(h^2) error of a
central difference; forward- and reverse-mode derivatives agree (dot-product
test).
"""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import euler_torch as ET
from paper_2402_05193_amd import workloads as WL

BCS = [(WL.PERIODIC,) * 6, (WL.ZERO_GRADIENT,) * 6, (WL.SYMMETRY,) * 6,
       (WL.PERIODIC, WL.PERIODIC, WL.ZERO_GRADIENT, WL.ZERO_GRADIENT, WL.SYMMETRY, WL.SYMMETRY)]


def case_state(bc, shape=(13, 11, 9), seed=3):
    case = WL.smooth_random(*shape, model=WL.EULER, seed=seed, bc=bc)
    oc = O.Config(**case.cfg_kwargs())
    return oc, O.prim_to_cons(oc, case.W)


@pytest.mark.parametrize("bc", BCS)
def test_forward_equals_c_oracle(bc):
    oc, U = case_state(bc)
    Ro = O.rhs(oc, U)
    Rt = ET.rhs(oc, torch.from_numpy(U)).numpy()
    assert np.abs(Rt - Ro).max() <= 5e-14 * np.abs(Ro).max()


def test_forward_equals_c_oracle_stiffened_gas_and_line():
    case = WL.smooth_random(40, 1, 1, model=WL.EULER, seed=9, bc=(WL.ZERO_GRADIENT,) * 6, gamma1=4.4, pinf1=6.0)
    oc = O.Config(**case.cfg_kwargs())
    U = O.prim_to_cons(oc, case.W)
    Ro = O.rhs(oc, U)
    Rt = ET.rhs(oc, torch.from_numpy(U)).numpy()
    assert np.abs(Rt - Ro).max() <= 5e-14 * np.abs(Ro).max()


def _dirs(U, seed, scale=1e-2):
    rng = np.random.default_rng(seed)
    v = torch.from_numpy(rng.standard_normal(U.shape) * np.abs(U).max(axis=(1, 2, 3), keepdims=True) * scale)
    w = torch.from_numpy(rng.standard_normal(U.shape))
    return v, w


def rough_state(bc, shape=(10, 9, 8), seed=1):
    """Independent random cell values: the face states differ by O(1), so the
    min/max branches of the wave speeds and the WENO weights are far from their
    kinks and the operator is smooth over small perturbations."""
    rng = np.random.default_rng(seed)
    nx, ny, nz = shape
    W = np.empty((5, nz, ny, nx))
    W[0] = 1 + 0.3 * rng.random((nz, ny, nx))
    W[1:4] = 0.3 * rng.standard_normal((3, nz, ny, nx))
    W[4] = 1 + 0.3 * rng.random((nz, ny, nx))
    oc = O.Config(nx=nx, ny=ny, nz=nz, dx=0.1, dy=0.1, dz=0.1, bc=bc)
    return oc, O.prim_to_cons(oc, W)


def fd_error(oc, Ut, v, w, exact, h):
    fd = float(((ET.rhs(oc, Ut + h * v) - ET.rhs(oc, Ut - h * v)) * w).sum()) / (2 * h)
    return abs(fd - exact) / abs(exact)


@pytest.mark.parametrize("bc", BCS[:2] + BCS[3:])
def test_vjp_matches_central_differences_second_order(bc):
    """<v, J^T w> against (<R(U + h v) - R(U - h v), w>) / 2h: error O(h^2) until round-off."""
    oc, U = rough_state(bc)
    Ut = torch.from_numpy(U)
    v, w = _dirs(U, 11, scale=1.0)
    exact = float((ET.rhs_vjp(oc, Ut, w) * v).sum())
    e5, e6 = fd_error(oc, Ut, v, w, exact, 1e-5), fd_error(oc, Ut, v, w, exact, 1e-6)
    assert e6 <= 1e-7
    assert e5 / e6 > 30.0


def test_vjp_matches_central_differences_symmetry_and_smooth():
    """Symmetry planes (mirror states give s* = 0 at the wall faces) and smooth
    fields (near-tied wave-speed candidates everywhere): a kink of the operator
    lies within larger perturbations, so only tiny ones are compared."""
    oc, U = rough_state(BCS[2])
    Ut = torch.from_numpy(U)
    v, w = _dirs(U, 12, scale=1.0)
    exact = float((ET.rhs_vjp(oc, Ut, w) * v).sum())
    assert fd_error(oc, Ut, v, w, exact, 1e-7) <= 1e-7
    oc, U = case_state(BCS[0], shape=(10, 9, 8), seed=5)
    Ut = torch.from_numpy(U)
    v, w = _dirs(U, 11, scale=1e-6)
    exact = float((ET.rhs_vjp(oc, Ut, w) * v).sum())
    assert fd_error(oc, Ut, v, w, exact, 1e-2) <= 1e-6


@pytest.mark.parametrize("bc", BCS)
def test_dot_product_forward_reverse(bc):
    oc, U = case_state(bc, seed=7)
    Ut = torch.from_numpy(U)
    v, w = _dirs(U, 13)
    a = float((ET.rhs_jvp(oc, Ut, v) * w).sum())
    b = float((v * ET.rhs_vjp(oc, Ut, w)).sum())
    assert abs(a - b) <= 1e-12 * max(abs(a), abs(b))


def test_rk3_step_vjp_matches_central_differences():
    oc, U = rough_state(BCS[0], shape=(9, 8, 7), seed=2)
    Ut = torch.from_numpy(U)
    dt = 0.4 * O.compute_dt(oc, U, 1.0)
    v, w = _dirs(U, 17, scale=1.0)
    exact = float((ET.rk3_step_vjp(oc, Ut, dt, w) * v).sum())
    h = 1e-7  # the stage states meet kinks of the operator for larger perturbations
    fd = float(((ET.rk3_step(oc, Ut + h * v, dt) - ET.rk3_step(oc, Ut - h * v, dt)) * w).sum()) / (2 * h)
    assert abs(fd - exact) <= 1e-7 * abs(exact)
    # and the step itself is the C oracle's
    Uo = O.rk3_step(oc, U, dt)
    assert np.abs(ET.rk3_step(oc, Ut, dt).numpy() - Uo).max() <= 1e-13 * np.abs(Uo).max()
