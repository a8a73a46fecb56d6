"""Tile-race check of the fused stage kernels, through the C ABI.

The library is built a second time with another tile shape (32 x 8 cells per
workgroup and 320 threads against 16 x 16 and 256: paper_2402_05193_amd.build,
libfvrk3_tile32x8.so).  Every x/y task list, the halo and ring assignments,
the rotation of the task remainder and the z chunks then map to threads
differently, while each cell's arithmetic does not depend on the tiling (the same
face fluxes from the same staged values, summed in the same order).  So both
builds must give bitwise the same results: a difference could only come from a
race on the LDS plane, the face buffers or the partial sums, or from a
tiling-dependent indexing mistake.  Cases: every model, both precisions, the
reconstruction variants, THINC, sixth-order viscous fluxes and a viscosity law,
ragged grids with mixed boundaries, single right-hand sides with their limiter
decisions on a shock-bubble state where the limiters act, and CFL-mode
trajectories.
"""
import os

import numpy as np
import pytest
import torch

from paper_2402_05193_amd import build as B
from paper_2402_05193_amd import solver as S
from paper_2402_05193_amd import workloads as WL

pytestmark = pytest.mark.gpu

MIXED_BC = (WL.PERIODIC, WL.PERIODIC, WL.ZERO_GRADIENT, WL.ZERO_GRADIENT, WL.SYMMETRY, WL.SYMMETRY)


@pytest.fixture(scope="module")
def tile_lib():
    if not os.path.exists(B.LIB_TILE):
        pytest.fail(f"{B.LIB_TILE} is missing: build it with `python -m paper_2402_05193_amd.build`")
    L = S.load(B.LIB_TILE)
    # the second build tiles differently: a 48 x 48 plane is 3 x 3 tiles of 16 x 16 and
    # 2 x 6 tiles of 32 x 8 (z chunks equal)
    probe = S.Config(nx=48, ny=48, nz=64, model=S.EULER)
    wg = both(L, lambda: S.stage_workgroups(probe))
    assert wg[0] * 12 == wg[1] * 9, wg
    return L


def state_of(cfg, case):
    W = torch.from_numpy(np.ascontiguousarray(case.W)).to("cuda", cfg.torch_dtype)
    U = torch.empty_like(W)
    S.prim_to_cons(cfg, W, U)
    return U


def both(tile_lib, fn):
    """fn() with the product library, then with the second tile shape."""
    a = fn()
    with S.using(tile_lib):
        b = fn()
    torch.cuda.synchronize()
    return a, b


def assert_bitwise(a, b, what):
    if not torch.equal(a, b):
        d = (a.double() - b.double()).abs().max().item()
        raise AssertionError(f"{what}: tile shapes differ (max abs difference {d:.3e})")


def cases():
    c = {
        "ns_tgv": (WL.taylor_green(40, viscous=True, ny=24, nz=20), {}),
        "euler_ragged": (WL.smooth_random(37, 19, 23, model=WL.EULER, seed=31, bc=MIXED_BC), {}),
        "ns_ragged_char": (WL.smooth_random(35, 17, 21, model=WL.NS, seed=32, bc=MIXED_BC, mu=0.02), dict(recon=1)),
        "ns_teno_visc6": (WL.taylor_green(36, viscous=True, ny=20, nz=18), dict(scheme=1, visc_order=6)),
        "ns_visc_law": (WL.taylor_green(33, viscous=True, ny=17, nz=19), dict(visc_law=2, T_ref=1.0,
                                                                             sutherland=0.4, gas_R=1.0)),
        "dim_ragged": (WL.smooth_random(34, 18, 22, model=WL.DIM, seed=33, bc=MIXED_BC, gamma1=6.12, pinf1=3.43,
                                        gamma2=1.4), {}),
        "dim_char_teno_thinc": (WL.shock_bubble(48, 24, 24), dict(thinc=1, scheme=1, recon=1)),
        "dim_thinc": (WL.interface_advection(40, axis=1), dict(thinc=1)),
    }
    return c


CASES = cases()


@pytest.mark.parametrize("dtype", [S.F64, S.F32])
@pytest.mark.parametrize("name", list(CASES))
def test_rhs_bitwise_across_tile_shapes(tile_lib, name, dtype):
    case, opts = CASES[name]
    cfg = S.config_from_case(case, dtype=dtype, **opts)
    U = state_of(cfg, case)
    wg = both(tile_lib, lambda: S.stage_workgroups(cfg))
    print(f"[tile-race] rhs {name} dtype {'f64' if dtype == S.F64 else 'f32'} shape {tuple(U.shape)} "
          f"workgroups 16x16: {wg[0]}, 32x8: {wg[1]}", flush=True)

    def run():
        R = torch.empty_like(U)
        S.rhs(cfg, U, R, dt=1e-3 * cfg.dx)
        return R

    Ra, Rb = both(tile_lib, run)
    assert torch.isfinite(Ra).all()
    assert_bitwise(Ra, Rb, f"rhs {name}")


@pytest.mark.parametrize("name", ["ns_tgv", "dim_ragged", "ns_teno_visc6", "dim_char_teno_thinc"])
def test_trajectory_bitwise_across_tile_shapes(tile_lib, name):
    """20 CFL steps (the fused stage-3 time-step reduction included)."""
    case, opts = CASES[name]
    cfg = S.config_from_case(case, cfl=0.5, **opts)
    U0 = state_of(cfg, case)
    print(f"[tile-race] 20 steps {name}", flush=True)

    def run():
        U = U0.clone()
        t = S.advance(cfg, U, 20, 0.0, S.workspace(cfg), t=0.0)
        return U, t

    (Ua, ta), (Ub, tb) = both(tile_lib, run)
    assert ta == tb, (ta, tb)
    assert_bitwise(Ua, Ub, f"20 steps {name}")


def test_limiter_decisions_bitwise_across_tile_shapes(tile_lib):
    """A 64 x 32 x 32 shock-bubble advanced 60 CFL steps on the GPU (past shock-bubble
    contact, where the positivity limiters act): R and every face's decision byte."""
    case = WL.shock_bubble(64, 32, 32)
    cfg = S.config_from_case(case, cfl=0.5, positivity=1)
    U = state_of(cfg, case)
    S.advance(cfg, U, 60, 0.0, S.workspace(cfg))
    dtd = torch.zeros(1, dtype=torch.float64, device="cuda")
    S.compute_dt(cfg, U, dtd, S.workspace(cfg))
    dt = float(dtd.item())
    print(f"[tile-race] shock-bubble 64x32x32 after 60 steps, dt {dt:.3e}", flush=True)

    def run():
        R, views = S.rhs_flags(cfg, U, torch.empty_like(U), dt=dt)
        return R, torch.cat([v.reshape(-1) for v in views])

    (Ra, fa), (Rb, fb) = both(tile_lib, run)
    nlim = int(torch.count_nonzero(fa))
    print(f"[tile-race] limited faces {nlim}", flush=True)
    assert nlim > 0
    assert torch.equal(fa, fb), "limiter decisions differ between tile shapes"
    assert_bitwise(Ra, Rb, "shock-bubble rhs with limiters")
