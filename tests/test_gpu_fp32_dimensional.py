"""FP32 on data in SI units, through the C ABI.

The paper runs its shock-bubble cases in single precision (Sec. 5.3, computations on
TPUs).  In SI units a shock's pressure jump is 1e4-1e9 Pa, so the WENO-Z smoothness
measure tau (the square of such a jump) divided by beta + eps (eps = 1e-30 in FP32)
exceeds the FP32 range wherever a candidate stencil is flat; the FP32 weights are
therefore evaluated scaled by the largest one (the same normalised weights).  These
tests run the air-helium shock-bubble (Ma 1.22, pressures ~1e5 Pa) and the
water-air shock tube (1e9 Pa against 1e5 Pa) in FP32 and compare them with the same
runs in FP64: every value finite, every state admissible, and the FP32 results within
FP32 round-off of FP64 where the scheme is a continuous function of the data (WENO5-Z),
except in the few cells next to a threshold decision (a positivity limiter at the
water-air interface) that FP32 rounding takes the other way.  TENO6-A switches candidate
stencils on a threshold everywhere, so only finiteness and admissibility are required there.
"""
import numpy as np
import pytest
import torch

from paper_2402_05193_amd import solver as S
from paper_2402_05193_amd import workloads as WL

pytestmark = pytest.mark.gpu

VARIANTS = {
    "weno": {},
    "weno_char": dict(recon=1),
    "teno": dict(scheme=1),
    "weno_thinc": dict(thinc=1),
}


def run(case, dtype, nsteps, **opts):
    cfg = S.config_from_case(case, dtype=dtype, cfl=0.5, **opts)
    W = torch.from_numpy(np.ascontiguousarray(case.W)).to("cuda", cfg.torch_dtype)
    U0 = torch.empty_like(W)
    S.prim_to_cons(cfg, W, U0)
    R = torch.empty_like(U0)
    S.rhs(cfg, U0, R, dt=1e-3 * cfg.dx)
    ws = S.workspace(cfg)
    U = U0.clone()
    t = S.advance(cfg, U, nsteps, 0.0, ws, t=0.0)
    rep = S.check_state(cfg, U, ws)
    torch.cuda.synchronize()
    return cfg, R.double(), U.double(), t, rep


def rel_diff(a, b):
    """|a_m - b_m| / max |b_m| per component and cell, the momentum components sharing the
    momentum vector's scale."""
    scale = [b[m].abs().max().item() for m in range(b.shape[0])]
    mom = max(scale[2:5])
    return torch.stack([(a[m] - b[m]).abs() / max(mom if 2 <= m <= 4 else scale[m], 1e-300)
                        for m in range(b.shape[0])])


def rel_by_component(a, b):
    """max |a_m - b_m| / max |b_m| per component (momenta sharing one scale)."""
    d = rel_diff(a, b)
    return [d[m].max().item() for m in range(d.shape[0])]


def cells_beyond(a, b, bar):
    """Cells where any component differs by more than bar (relative), and where they lie."""
    far = (rel_diff(a, b) > bar).any(dim=0)
    return int(far.sum()), far.nonzero().tolist()[:8]


@pytest.mark.parametrize("variant", list(VARIANTS))
def test_shock_bubble_si_units_fp32(variant):
    case = WL.shock_bubble(64, 32, 32)
    opts = VARIANTS[variant]
    print(f"[fp32-si] shock-bubble 64x32x32 {variant}", flush=True)
    _, R64, U64, t64, _ = run(case, S.F64, 20, **opts)
    _, R32, U32, t32, rep = run(case, S.F32, 20, **opts)
    assert torch.isfinite(R32).all(), "FP32 right-hand side not finite"
    assert torch.isfinite(U32).all(), "FP32 state not finite after 20 steps"
    assert rep.status == S.OK, f"FP32 state not admissible: status {rep.status}, first bad cell {rep.first_bad_cell}"
    rr = rel_by_component(R32, R64)
    ru = rel_by_component(U32, U64)
    print(f"[fp32-si] R rel {max(rr):.2e} U rel after 20 steps {max(ru):.2e} t {t32:.6e} / {t64:.6e}", flush=True)
    # one RHS: helium traces (alpha ~ 1e-8) at the shock set the largest relative
    # differences (alpha1 rho1, measured <= 9.2e-4); WENO5-Z states after 20 steps
    # measured <= 4.4e-5, the simulated time <= 4e-7 relative
    assert max(rr) <= 5e-3, rr
    if not opts.get("scheme"):
        nfar, where = cells_beyond(U32, U64, 1e-4)
        print(f"[fp32-si] cells beyond 1e-4: {nfar} of {U64[0].numel()} {where}", flush=True)
        assert max(ru) <= 5e-2, ru
        assert nfar <= U64[0].numel() // 1000, (nfar, where)
        assert abs(t32 - t64) <= 1e-5 * t64


@pytest.mark.parametrize("variant", ["weno", "teno"])
def test_water_air_tube_fp32(variant):
    """Water at 1e9 Pa against air at 1e5 Pa, limiters on, 100 CFL steps."""
    case = WL.air_water_tube(200)
    opts = VARIANTS[variant]
    print(f"[fp32-si] water-air tube 200 {variant}", flush=True)
    _, R64, U64, t64, _ = run(case, S.F64, 100, positivity=1, **opts)
    _, R32, U32, t32, rep = run(case, S.F32, 100, positivity=1, **opts)
    assert torch.isfinite(R32).all() and torch.isfinite(U32).all()
    assert rep.status == S.OK, f"FP32 state not admissible: status {rep.status}, first bad cell {rep.first_bad_cell}"
    ru = rel_by_component(U32, U64)
    print(f"[fp32-si] U rel after 100 steps {max(ru):.2e} {['%.1e' % x for x in ru]} t {t32:.6e} / {t64:.6e}",
          flush=True)
    if variant == "weno":
        nfar, where = cells_beyond(U32, U64, 1e-4)
        print(f"[fp32-si] cells beyond 1e-4: {nfar} of {U64[0].numel()} {where}", flush=True)
        assert max(ru) <= 5e-2, ru
        assert nfar <= 2, (nfar, where)
