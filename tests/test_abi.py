"""The C-ABI library loads and exports every entry point of include/fvrk3.h;
host-side validation returns the documented codes (no GPU needed: every case
here fails before any HIP call)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fvrk3.h")

S = pytest.importorskip("paper_2402_05193_amd.solver")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|int32_t|const char\*|size_t)\s+(\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_boundary():
    fns = header_functions()
    for name in ("init_state", "rhs", "rk3_step", "advance", "rhs_adjoint", "rk3_stage", "prim_to_cons",
                 "workspace_bytes", "check_state", "last_error", "compute_dt"):
        assert name in fns


def test_library_exports_every_declared_symbol():
    L = S.lib()
    for name in header_functions():
        assert hasattr(L, name), name
        assert ctypes.cast(getattr(L, name), ctypes.c_void_p).value


def test_tile_variant_exports_every_declared_symbol():
    """The build with the second tile shape (the GPU tile-race check) is the same
    boundary; its host-side validation answers like the product's."""
    from paper_2402_05193_amd import build as B
    L = S.load(B.LIB_TILE)
    for name in header_functions():
        assert ctypes.cast(getattr(L, name), ctypes.c_void_p).value, name
    with S.using(L):
        assert call_rhs(cfg(nx=0)) == S.EINVAL
    assert S.lib() is not L


def cfg(**kw):
    base = dict(nx=8, ny=8, nz=8, dx=0.1, dy=0.1, dz=0.1)
    base.update(kw)
    return S.Config(**base)


def call_rhs(c, U=256, R=512, dt=0.0):
    cs = c.c_struct()
    return S.lib().rhs(ctypes.byref(cs), U, R, dt, None)


def test_validation_codes():
    assert call_rhs(cfg(nx=0)) == S.EINVAL
    assert call_rhs(cfg(model=7)) == S.EINVAL
    assert call_rhs(cfg(dtype=3)) == S.EINVAL
    assert call_rhs(cfg(dx=-1.0)) == S.EINVAL
    assert call_rhs(cfg(gamma1=1.0)) == S.EINVAL
    assert call_rhs(cfg(bc=(S.PERIODIC, S.ZERO_GRADIENT) + (S.PERIODIC,) * 4)) == S.EINVAL
    assert call_rhs(cfg(nx=2, bc=(S.SYMMETRY,) * 2 + (S.PERIODIC,) * 4)) == S.EINVAL
    assert call_rhs(cfg(), U=None) == S.ENULL
    assert call_rhs(cfg(), U=264) == S.EALIGN
    assert call_rhs(cfg(), U=256, R=256) == S.EINVAL
    assert call_rhs(cfg(), dt=float("nan")) == S.EINVAL
    assert "dt" in S.last_error()
    assert call_rhs(cfg(scheme=2)) == S.EINVAL
    assert "scheme" in S.last_error()
    assert call_rhs(cfg(recon=2)) == S.EINVAL
    assert call_rhs(cfg(visc_order=5)) == S.EINVAL
    assert call_rhs(cfg(visc_order=6)) == S.EINVAL            # sixth order is for the viscous model
    assert call_rhs(cfg(model=S.NS, mu=0.01, visc_order=6)) == S.EUNSUPPORTED   # needs rhs_ws
    assert "rhs_ws" in S.last_error()
    c6 = cfg(model=S.NS, mu=0.01, visc_order=6).c_struct()
    assert S.lib().rk3_stage(ctypes.byref(c6), 1, 256, 256, 512, 1e-3, None, None) == S.EUNSUPPORTED
    assert S.lib().rhs_ws(ctypes.byref(c6), 256, 512, 0.0, None, None) == S.ENULL
    c = cfg().c_struct()
    c.abi_version = 99
    assert S.lib().rhs(ctypes.byref(c), 256, 512, 0.0, None) == S.EINVAL
    assert "abi_version" in S.last_error()
    assert S.lib().rhs(None, 256, 512, 0.0, None) == S.ENULL


def test_stage_and_step_validation():
    c = cfg().c_struct()
    L = S.lib()
    assert L.rk3_stage(ctypes.byref(c), 4, 256, 256, 512, 1e-3, None, None) == S.EINVAL
    assert L.rk3_stage(ctypes.byref(c), 1, 256, 768, 512, 1e-3, None, None) == S.EINVAL  # stage 1 needs Uk == Un
    assert L.rk3_stage(ctypes.byref(c), 2, 256, 512, 512, 1e-3, None, None) == S.EINVAL  # Uout aliases Uk
    assert L.rk3_stage(ctypes.byref(c), 2, 256, 512, 768, 0.0, None, None) == S.EINVAL  # dt <= 0
    assert L.rk3_step(ctypes.byref(c), 256, 1e-3, None, None) == S.ENULL
    assert L.advance(ctypes.byref(c), 256, -1, 1e-3, None, 512, None) == S.EINVAL
    c2 = cfg(cfl=0.0).c_struct()
    assert L.advance(ctypes.byref(c2), 256, 3, 0.0, None, 512, None) == S.EINVAL
    # the adjoint covers single-phase Euler, FP64, limiters off
    for bad in (cfg(model=S.NS, mu=0.01), cfg(model=S.DIM), cfg(dtype=S.F32), cfg(positivity=1), cfg(recon=1),
                cfg(scheme=1)):
        cb = bad.c_struct()
        assert L.rhs_adjoint(ctypes.byref(cb), 256, 512, 768, None, None) == S.EUNSUPPORTED
        assert L.rk3_step_adjoint(ctypes.byref(cb), 256, 512, 1e-3, 768, None) == S.EUNSUPPORTED
        assert L.rk3_step_adjoint_stages(ctypes.byref(cb), 256, 320, 384, 512, 1e-3, 768, None) == S.EUNSUPPORTED
    assert L.rhs_adjoint(ctypes.byref(c), 256, 512, 256, None, None) == S.EINVAL    # Ubar aliases U
    assert L.rhs_adjoint(ctypes.byref(c), 256, None, 768, None, None) == S.ENULL
    assert L.rk3_step_adjoint(ctypes.byref(c), 256, 512, 0.0, 768, None) == S.EINVAL  # dt <= 0
    assert L.rk3_step_adjoint(ctypes.byref(c), 256, 512, 1e-3, None, None) == S.ENULL
    assert L.rk3_step_adjoint_stages(ctypes.byref(c), 256, None, 384, 512, 1e-3, 768, None) == S.ENULL  # U1
    assert L.rk3_step_adjoint_stages(ctypes.byref(c), 256, 320, 384, 320, 1e-3, 768, None) == S.EINVAL  # Ubar = U1
    assert L.rk3_step_adjoint_stages(ctypes.byref(c), 256, 320, 384, 512, 0.0, 768, None) == S.EINVAL  # dt <= 0
    assert L.init_state(ctypes.byref(c), 99, None, 0, 0, 256, None) == S.EINVAL
    p = (ctypes.c_double * 2)(0.1, 1.0)
    assert L.init_state(ctypes.byref(c), S.CASE_TGV, p, 2, 0, 256, None) == S.EINVAL  # too few params


def test_workspace_and_ncomp():
    c6 = cfg(nx=10, ny=3, nz=2, model=S.NS, mu=0.01, visc_order=6)
    a256 = lambda b: (b + 255) // 256 * 256
    npad, n = 16 * 9 * 8, 60
    assert S.workspace_bytes(c6) == 2 * a256(8 * 5 * n) + 256 + a256(4 * npad * 8) + a256(9 * npad * 8) + \
        a256(4 * n * 8)
    c = cfg(nx=10, ny=3, nz=2)
    state = 8 * 5 * 60
    pad = (state + 255) // 256 * 256
    assert S.workspace_bytes(c) == 2 * pad + 256
    assert S.ncomp(c) == 5
    assert S.ncomp(cfg(model=S.DIM)) == 7
    assert S.workspace_bytes(cfg(dtype=S.F32)) == 2 * ((4 * 5 * 512 + 255) // 256 * 256) + 256
    out = ctypes.c_size_t(0)
    cs = c.c_struct()
    assert S.lib().adjoint_workspace_bytes(ctypes.byref(cs), ctypes.byref(out)) == S.OK
    assert out.value == 5 * pad


def test_advance_noalloc_rejects_problems_beyond_its_scratch():
    """advance_noalloc checks the workspace size before any device work."""
    c = cfg(nx=256, ny=256, nz=256, model=S.NS, mu=1e-3)
    cs = c.c_struct()
    assert S.workspace_bytes(c) > S.NOALLOC_SCRATCH_BYTES
    assert S.lib().advance_noalloc(ctypes.byref(cs), 256, 1, 1e-3, None) == S.EINVAL
    assert "scratch" in S.last_error()


def test_noalloc_scratch_size_matches_header():
    text = open(HEADER).read()
    m = re.search(r"#define FV_NOALLOC_SCRATCH_BYTES \((\d+)ull << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == S.NOALLOC_SCRATCH_BYTES
