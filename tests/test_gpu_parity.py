"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Both sides receive the same conservative state: the seeded primitive field of
paper_2402_05193_amd.workloads converted by the oracle.  Bar (FP64): per
component, max|R_gpu - R_oracle| / max|R_oracle| <= 1e-12 for one RHS, and
max|U_gpu - U_oracle| / max|U_oracle| <= 1e-10 after 100 TVD-RK3 steps.
"""
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_2402_05193_amd import solver as S
from paper_2402_05193_amd import workloads as WL

pytestmark = pytest.mark.gpu

RHS_TOL = 1e-12
STEP_TOL = 1e-10


def dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def host(t):
    torch.cuda.synchronize()
    return t.detach().to("cpu", torch.float64).numpy()


def comp_rel(gpu, ref):
    """Per-component max abs difference over max abs reference.  Momentum
    components share the momentum vector's scale (a component that vanishes by
    symmetry has only round-off as its own reference)."""
    nc = ref.shape[0]
    g = gpu.reshape(nc, -1)
    r = ref.reshape(nc, -1)
    v0 = 2 if nc == 7 else 1
    mom = np.abs(r[v0:v0 + 3]).max()
    scale_all = np.abs(r).max()
    out = []
    for m in range(nc):
        s = np.abs(r[m]).max()
        if v0 <= m < v0 + 3:
            s = mom
        if s < 1e-300:
            s = scale_all
        out.append(np.abs(g[m] - r[m]).max() / s)
    return np.array(out)


def roundoff_floor(oc, U, dt, cells=None, trials=2, seed=1):
    """The oracle's own round-off floor of the case, per component: the largest of
    (1) the relative change of its R when every input value moves by one unit in
    the last place (random sign; the conditioning of the problem: in low-Mach flow
    the pressure flux ~1/(gamma Ma^2) cancels in the flux difference, so this can
    exceed 1e-12), (2) the difference between the oracle and the same source built
    with multiply-add contraction (every intermediate rounded differently), and
    (3) the difference when every exp / pow / tanh / atanh / cosh / sinh result is
    one ulp higher (the two sides use different math libraries; THINC's interface
    normal differences psi = alpha^0.1 / (...) of neighbouring cells, where such an
    ulp is amplified)."""
    rng = np.random.default_rng(seed)
    R = O.rhs(oc, U, dt=dt) if cells is None else O.rhs_cells(oc, U, cells, dt=dt)
    worst = np.zeros(U.shape[0])
    for _ in range(trials):
        Up = U * (1.0 + rng.choice([-1.0, 1.0], size=U.shape) * 2.0 ** -53)
        Rp = O.rhs(oc, Up, dt=dt) if cells is None else O.rhs_cells(oc, Up, cells, dt=dt)
        worst = np.maximum(worst, comp_rel(Rp, R))
    for kind in ("fma", "ulp"):
        with O.variant(kind):
            Rc = O.rhs(oc, U, dt=dt) if cells is None else O.rhs_cells(oc, U, cells, dt=dt)
        worst = np.maximum(worst, comp_rel(Rc, R))
    return worst


def oracle_cfg(case, **kw):
    d = case.cfg_kwargs()
    d.update(kw)
    return O.Config(**d)


def solver_cfg(case, dtype=S.F64, **kw):
    return S.config_from_case(case, dtype=dtype, **kw)


MIXED_BC = (WL.PERIODIC, WL.PERIODIC, WL.ZERO_GRADIENT, WL.ZERO_GRADIENT, WL.SYMMETRY, WL.SYMMETRY)


def cases():
    return {
        "euler_tgv32": WL.taylor_green(32),
        "euler_ragged": WL.smooth_random(13, 11, 9, model=WL.EULER, seed=21, bc=MIXED_BC),
        "euler_line": WL.gauss_wave(64, axis=0),
        "euler_plane": WL.smooth_random(20, 17, 1, model=WL.EULER, seed=4),
        "ns_tgv32": WL.taylor_green(32, viscous=True),
        "ns_ragged": WL.smooth_random(19, 13, 10, model=WL.NS, seed=22, bc=MIXED_BC, mu=0.02, prandtl=0.7),
        "dim_smooth": WL.smooth_random(12, 10, 9, model=WL.DIM, seed=23, gamma1=1.66, gamma2=1.4),
        "dim_ragged": WL.smooth_random(17, 9, 7, model=WL.DIM, seed=24, bc=MIXED_BC, gamma1=6.12, pinf1=3.43,
                                       gamma2=1.4),
        "dim_sbi": WL.shock_bubble(48, 24, 24),
    }


@pytest.fixture(scope="module")
def all_cases():
    return cases()


@pytest.mark.parametrize("name", list(cases().keys()))
def test_rhs_parity(all_cases, name):
    case = all_cases[name]
    oc = oracle_cfg(case)
    U = O.prim_to_cons(oc, case.W)
    dt = 0.3 * O.compute_dt(oc, U, 1.0)
    print(f"[parity] rhs {name} shape={U.shape} dt={dt:.3e}", flush=True)
    Ro = O.rhs(oc, U, dt=dt)
    sc = solver_cfg(case)
    Ud = dev(U)
    Rd = torch.empty_like(Ud)
    S.rhs(sc, Ud, Rd, dt=dt)
    err = comp_rel(host(Rd), Ro)
    floor = roundoff_floor(oc, U, dt)
    tol = np.maximum(RHS_TOL, 2.0 * floor)
    print(f"[parity] rhs {name} rel err {np.array2string(err, precision=2)} "
          f"round-off floor {np.array2string(floor, precision=2)}", flush=True)
    assert np.all(err <= tol), (err, floor)


def test_prim_to_cons_parity(all_cases):
    for name, case in all_cases.items():
        oc = oracle_cfg(case)
        sc = solver_cfg(case)
        Uo = O.prim_to_cons(oc, case.W)
        Ud = S.prim_to_cons(sc, dev(case.W), S.empty_state(sc))
        assert np.all(comp_rel(host(Ud), Uo) <= 1e-15), name
        Wd = S.cons_to_prim(sc, dev(Uo), S.empty_state(sc))
        assert np.all(comp_rel(host(Wd), case.W) <= 1e-14), name


def test_init_state_tgv_matches_generator():
    case = WL.taylor_green(24, seed=2402)
    sc = solver_cfg(case)
    Ud = S.init_state(sc, S.CASE_TGV, [0.1, 1.0, 1e-3], S.empty_state(sc), seed=2402)
    Uo = O.prim_to_cons(oracle_cfg(case), case.W)
    assert np.all(comp_rel(host(Ud), Uo) <= 1e-14)


def test_init_state_convergence_cases():
    """The convergence test's Gaussian density wave (exact cell averages, along each
    axis) and the isentropic vortex (5 x 5 Gauss cell averages) against the host
    generators."""
    for axis in range(3):
        case = WL.gauss_wave(64, axis=axis)
        sc = solver_cfg(case)
        Ud = S.init_state(sc, S.CASE_GAUSS_WAVE, [axis, 1.0, 1.0], S.empty_state(sc))
        Uo = O.prim_to_cons(oracle_cfg(case), case.W)
        assert np.all(comp_rel(host(Ud), Uo) <= 1e-14), axis
    from test_oracle_accuracy import _vortex_cell_averages
    n = 32
    h = 10.0 / n
    sc = S.Config(nx=n, ny=n, nz=1, dx=h, dy=h, dz=h)
    Ud = S.init_state(sc, S.CASE_ISENTROPIC_VORTEX, [5.0, 5.0, 5.0, 1.0, 1.0], S.empty_state(sc))
    assert np.all(comp_rel(host(Ud), _vortex_cell_averages(n, 0.0)) <= 1e-14)


def test_init_state_sbi_matches_generator():
    case = WL.shock_bubble(32, 16, 16)
    sc = solver_cfg(case)
    rho2, u2, p2 = case.meta["post_shock"]
    H = case.meta["H"]
    params = [0.060, 0.090, H / 2, H / 2, 0.25 * H, WL.ALPHA_EPS, rho2, u2, p2, 1.2041, 101325.0, 0.1660]
    Ud = S.init_state(sc, S.CASE_SBI, params, S.empty_state(sc))
    Uo = O.prim_to_cons(oracle_cfg(case), case.W)
    assert np.all(comp_rel(host(Ud), Uo) <= 1e-14)


def test_uniform_state_exactly_preserved():
    for model, state, extra in [(WL.EULER, (1.3, 0.3, -0.2, 0.1, 2.0), {}),
                                (WL.NS, (1.3, 0.3, -0.2, 0.1, 2.0), dict(mu=0.01)),
                                (WL.DIM, (0.4, 0.35, 0.3, -0.2, 0.1, 2.0, 0.45), dict(gamma1=1.66))]:
        for bc in (WL.PERIODIC, WL.ZERO_GRADIENT):
            case = WL.uniform(23, 18, 13, model=model, state=state, bc=(bc,) * 6, h=(0.1, 0.2, 0.3), **extra)
            sc = solver_cfg(case)
            U = dev(O.prim_to_cons(oracle_cfg(case), case.W))
            R = torch.empty_like(U)
            S.rhs(sc, U, R, dt=1e-3)
            assert int(torch.count_nonzero(R)) == 0, (model, bc)


def test_large_grid_component_offsets():
    """Element offsets beyond 2^31 (1024 x 1024 x 416 cells, five FP64 components,
    17 GB per state): a uniform state with distinct component values gives R = 0
    exactly and a first RK stage that returns the state bit for bit (a component
    read from the wrong offset would break the uniformity)."""
    small = WL.uniform(2, 2, 2, model=WL.NS, state=(1.3, 0.3, -0.2, 0.1, 2.0), mu=0.01)
    u0 = O.prim_to_cons(oracle_cfg(small), small.W)[:, 0, 0, 0]
    sc = solver_cfg(small, nx=1024, ny=1024, nz=416)
    assert sc.ncells * sc.ncomp > 2 ** 31
    print(f"[parity] large grid {sc.nx}x{sc.ny}x{sc.nz}", flush=True)
    U = torch.empty((sc.ncomp, sc.nz, sc.ny, sc.nx), dtype=torch.float64, device="cuda")
    for m in range(sc.ncomp):
        U[m].fill_(float(u0[m]))
    R = torch.empty_like(U)
    S.rhs(sc, U, R, dt=1e-3)
    assert int(torch.count_nonzero(R)) == 0
    del R
    U1 = torch.empty_like(U)
    S.rk3_stage(sc, 1, U, U, U1, 1e-3)
    assert torch.equal(U1, U)
    del U, U1
    torch.cuda.empty_cache()

def test_conservation_on_gpu():
    for model, extra in [(WL.EULER, {}), (WL.NS, dict(mu=0.01)), (WL.DIM, dict(gamma1=1.66))]:
        case = WL.smooth_random(37, 29, 21, model=model, seed=31, **extra)
        sc = solver_cfg(case)
        U = dev(O.prim_to_cons(oracle_cfg(case), case.W))
        R = torch.empty_like(U)
        S.rhs(sc, U, R, dt=1e-4)
        Rh = host(R).reshape(sc.ncomp, -1)
        for m in range(6 if model == WL.DIM else 5):
            assert abs(Rh[m].sum()) <= 1e-13 * np.abs(Rh[m]).sum(), (model, m)


def test_mirror_symmetry_on_gpu():
    case = WL.smooth_random(21, 18, 15, model=WL.NS, seed=5, bc=(WL.ZERO_GRADIENT,) * 6, mu=0.01)
    sc = solver_cfg(case)
    U = O.prim_to_cons(oracle_cfg(case), case.W)
    R = host(S.rhs(sc, dev(U), S.empty_state(sc)))
    for axis in range(3):
        Um = np.flip(U, axis=3 - axis).copy()
        Um[1 + axis] *= -1
        Rm = host(S.rhs(sc, dev(Um), S.empty_state(sc)))
        ref = np.flip(R, axis=3 - axis).copy()
        ref[1 + axis] *= -1
        assert np.all(comp_rel(Rm, ref) <= 1e-13), axis


def test_determinism():
    case = WL.shock_bubble(40, 20, 20)
    sc = solver_cfg(case)
    U = dev(O.prim_to_cons(oracle_cfg(case), case.W))
    R1 = S.rhs(sc, U, torch.empty_like(U), dt=1e-7)
    R2 = S.rhs(sc, U, torch.empty_like(U), dt=1e-7)
    assert torch.equal(R1, R2)


@pytest.mark.parametrize("name", ["euler_tgv32", "ns_ragged", "dim_smooth"])
def test_rk3_step_parity(all_cases, name):
    case = all_cases[name]
    oc = oracle_cfg(case)
    U = O.prim_to_cons(oc, case.W)
    dt = 0.5 * O.compute_dt(oc, U, 1.0)
    sc = solver_cfg(case)
    Ud = dev(U)
    # stages one by one through rk3_stage, and the whole step through rk3_step
    A = torch.empty_like(Ud)
    B = torch.empty_like(Ud)
    C = torch.empty_like(Ud)
    S.rk3_stage(sc, 1, Ud, Ud, A, dt)
    S.rk3_stage(sc, 2, Ud, A, B, dt)
    S.rk3_stage(sc, 3, Ud, B, C, dt)
    U1 = O.rk3_stage(oc, 1, U, U, dt)
    U2 = O.rk3_stage(oc, 2, U, U1, dt)
    U3 = O.rk3_stage(oc, 3, U, U2, dt)
    for g, o in ((A, U1), (B, U2), (C, U3)):
        assert np.all(comp_rel(host(g), o) <= 1e-13)
    ws = S.workspace(sc)
    D = Ud.clone()
    S.rk3_step(sc, D, dt, ws)
    assert torch.equal(D, C)


def test_hundred_steps_c1():
    case = WL.taylor_green(32)
    oc = oracle_cfg(case)
    U = O.prim_to_cons(oc, case.W)
    print("[parity] 100 steps TGV 32^3 oracle ...", flush=True)
    Uo, t_o = O.advance(oc, U, 100, dt=1e-3)
    sc = solver_cfg(case)
    Ud = dev(U)
    ws = S.workspace(sc)
    t = S.advance(sc, Ud, 100, 1e-3, ws, t=0.0)
    assert t == pytest.approx(t_o, rel=1e-15)
    err = comp_rel(host(Ud), Uo)
    print(f"[parity] 100 steps rel err {err}", flush=True)
    assert np.all(err <= STEP_TOL), err


def test_hundred_steps_ns_tgv64():
    """The viscous benchmark case at 64^3: 100 CFL-0.5 steps of the GPU against the
    oracle (spec bar 1e-10 per component after 100 steps) and the simulated time."""
    case = WL.taylor_green(64, viscous=True)
    oc = oracle_cfg(case)
    U = O.prim_to_cons(oc, case.W)
    print("[parity] 100 CFL steps NS TGV 64^3 oracle ...", flush=True)
    Uo, t_o = O.advance(oc, U, 100, dt=0.0, cfl=0.5)
    sc = solver_cfg(case, cfl=0.5)
    Ud = dev(U)
    t = S.advance(sc, Ud, 100, 0.0, S.workspace(sc), t=0.0)
    err = comp_rel(host(Ud), Uo)
    print(f"[parity] NS TGV 64^3 100 steps rel err {np.array2string(err, precision=2)}, time {t:.12e} "
          f"vs {t_o:.12e}", flush=True)
    assert t == pytest.approx(t_o, rel=1e-13)
    assert np.all(err <= STEP_TOL), err


def test_cfl_dt_and_advance_parity():
    case = WL.taylor_green(24, viscous=True, reynolds=50.0)
    oc = oracle_cfg(case)
    U = O.prim_to_cons(oc, case.W)
    sc = solver_cfg(case, cfl=0.5)
    Ud = dev(U)
    ws = S.workspace(sc)
    dtd = torch.zeros(1, dtype=torch.float64, device="cuda")
    S.compute_dt(sc, Ud, dtd, ws)
    assert float(dtd.item()) == pytest.approx(O.compute_dt(oc, U, 0.5), rel=1e-14)
    Uo, to = O.advance(oc, U, 5, dt=0.0, cfl=0.5)
    t = S.advance(sc, Ud, 5, 0.0, ws, t=0.0)
    assert t == pytest.approx(to, rel=1e-13)
    assert np.all(comp_rel(host(Ud), Uo) <= 1e-12)


def test_fused_stage3_cfl_matches_stage_and_oracle_dt():
    case = WL.taylor_green(24, viscous=True, reynolds=50.0)
    oc = oracle_cfg(case)
    U = O.prim_to_cons(oc, case.W)
    sc = solver_cfg(case, cfl=0.5)
    Ud = dev(U)
    ws = S.workspace(sc)
    dtd = torch.full((1,), 1e-3, dtype=torch.float64, device="cuda")
    A = torch.empty_like(Ud)
    B = torch.empty_like(Ud)
    C = torch.empty_like(Ud)
    S.rk3_stage(sc, 1, Ud, Ud, A, 0.0, dtd)
    S.rk3_stage(sc, 2, Ud, A, B, 0.0, dtd)
    S.rk3_stage(sc, 3, Ud, B, C, 0.0, dtd)
    D = torch.empty_like(Ud)
    nxt = torch.zeros(1, dtype=torch.float64, device="cuda")
    S.rk3_stage3_cfl(sc, Ud, B, D, dtd, nxt, ws)
    assert torch.equal(C, D)
    assert float(nxt.item()) == pytest.approx(O.compute_dt(oc, host(D), 0.5), rel=1e-14)
    # in place (stage 3 overwrites U^n) and dt_next aliasing dt_dev
    E = Ud.clone()
    S.rk3_stage3_cfl(sc, E, B, E, dtd, dtd, ws)
    assert torch.equal(E, C)
    assert float(dtd.item()) == float(nxt.item())


def test_check_state_reports_bad_cells():
    case = WL.taylor_green(16)
    sc = solver_cfg(case)
    U = dev(O.prim_to_cons(oracle_cfg(case), case.W))
    ws = S.workspace(sc)
    assert S.check_state(sc, U, ws).status == S.OK
    V = U.clone()
    V[0, 3, 2, 1] = -1.0
    rep = S.check_state(sc, V, ws)
    assert rep.status == S.EINADMISSIBLE and rep.first_bad_cell == (3 * 16 + 2) * 16 + 1 and rep.bad_count_clamped == 1
    V[4, 0, 0, 5] = float("nan")
    rep = S.check_state(sc, V, ws)
    assert rep.status == S.ENONFINITE and rep.first_bad_cell == 5 and rep.bad_count_clamped == 2


def test_fp32_error_against_fp64_oracle():
    for name, case in [("euler_tgv32", WL.taylor_green(32)), ("ns_tgv32", WL.taylor_green(32, viscous=True)),
                       ("dim_smooth", WL.smooth_random(12, 10, 9, model=WL.DIM, seed=23, gamma1=1.66))]:
        oc = oracle_cfg(case)
        U = O.prim_to_cons(oc, case.W)
        Ro = O.rhs(oc, U, dt=1e-4)
        sc = solver_cfg(case, dtype=S.F32)
        Ud = dev(U, torch.float32)
        Rd = S.rhs(sc, Ud, torch.empty_like(Ud), dt=1e-4)
        err = comp_rel(host(Rd), Ro)
        print(f"[fp32] rhs {name} rel err per component {err}", flush=True)
        # single-precision rounding of the inputs alone costs ~1e-7 U / (dx R)
        assert np.all(err < 5e-3), err



def test_fp32_trajectory_error_statement():
    """FP32 against FP64 over the NS TGV's 200 CFL steps (the C2 step count) at 32^3:
    the FP64 path is the oracle's to round-off (tests above), so this states the FP32
    trajectory's own error; measured ~1e-5 per component and 4e-6 in kinetic energy
    (the same at 128^3)."""
    case = WL.taylor_green(32, viscous=True, with_field=False)
    res = {}
    for dt_ in (S.F64, S.F32):
        c64 = solver_cfg(case)
        U0 = S.init_state(c64, S.CASE_TGV, [0.1, 1.0, 1e-3], S.empty_state(c64), seed=2402)
        cfg = solver_cfg(case, dtype=dt_)
        U = U0.to(torch.float32) if dt_ == S.F32 else U0
        t = S.advance(cfg, U, 200, 0.0, S.workspace(cfg), t=0.0)
        res[dt_] = (host(U), t)
    (U64, t64), (U32, t32) = res[S.F64], res[S.F32]
    err = comp_rel(U32, U64)
    ke = [float((0.5 * (u[1] ** 2 + u[2] ** 2 + u[3] ** 2) / u[0]).mean()) for u in (U64, U32)]
    print(f"[fp32] tgv32 200 steps: state rel err {np.array2string(err, precision=2)}, kinetic energy "
          f"{abs(ke[1] - ke[0]) / ke[0]:.2e}, time {abs(t32 - t64) / t64:.2e}", flush=True)
    assert np.all(err < 5e-5), err
    assert abs(ke[1] - ke[0]) < 2e-5 * ke[0]
    assert abs(t32 - t64) < 1e-5 * t64

FULL_OPTS = {
    "": {},
    "char": dict(recon=1),
    "teno": dict(scheme=1),
    "single_phase_setup": dict(scheme=1, visc_order=6),    # TENO6-A + sixth-order viscous fluxes
    "thinc": dict(thinc=1),
    "char_teno_thinc": dict(scheme=1, recon=1, thinc=1),
}


@pytest.mark.parametrize("cfgname,opt", [("ns_tgv_256", ""), ("dim_sbi_256x128x128", ""), ("ns_tgv_256", "char"),
                                         ("ns_tgv_256", "teno"), ("ns_tgv_256", "single_phase_setup"),
                                         ("dim_sbi_256x128x128", "thinc"),
                                         ("dim_sbi_256x128x128", "char_teno_thinc")])
def test_full_size_sampled_parity(cfgname, opt):
    """The benchmark's full-size workloads (and their f3/f4 variants) in the
    launch configuration the benchmark times, on sampled cells."""
    kw = FULL_OPTS[opt]
    if cfgname == "ns_tgv_256":
        case = WL.taylor_green(256, viscous=True, with_field=False)
        sc = solver_cfg(case, **kw)
        U = S.init_state(sc, S.CASE_TGV, [0.1, 1.0, 1e-3], S.empty_state(sc), seed=2402)
        dt = 1e-3
    else:
        case = WL.shock_bubble(256, 128, 128, with_field=False)
        sc = solver_cfg(case, **kw)
        rho2, u2, p2 = case.meta["post_shock"]
        H = case.meta["H"]
        params = [0.060, 0.090, H / 2, H / 2, 0.25 * H, WL.ALPHA_EPS, rho2, u2, p2, 1.2041, 101325.0, 0.1660]
        U = S.init_state(sc, S.CASE_SBI, params, S.empty_state(sc))
        dt = 2e-7
    print(f"[parity] full size {cfgname} {opt}", flush=True)
    R = S.rhs(sc, U, torch.empty_like(U), dt=dt)
    U1 = None
    if sc.visc_order != 6:   # rk3_stage has no workspace for the sixth-order passes
        U1 = torch.empty_like(U)
        S.rk3_stage(sc, 1, U, U, U1, dt)
    torch.cuda.synchronize()
    Uh = host(U)
    Rh = host(R).reshape(sc.ncomp, -1)
    U1h = host(U1).reshape(sc.ncomp, -1) if U1 is not None else None
    del R, U1, U
    torch.cuda.empty_cache()
    rng = np.random.default_rng(7)
    n = sc.ncells
    cells = np.concatenate([rng.integers(0, n, 300), [0, n - 1, sc.nx - 1, sc.nx * sc.ny - 1]])
    if cfgname.startswith("dim"):
        # a line of cells through the shock and the bubble centre
        k = sc.nz // 2
        j = sc.ny // 2
        xs = np.arange(sc.nx)
        cells = np.concatenate([cells, (k * sc.ny + j) * sc.nx + xs[::3]])
    oc = oracle_cfg(case, **kw)
    Ro = O.rhs_cells(oc, Uh, cells, dt=dt)
    Rg = Rh[:, cells]
    err = comp_rel(Rg, Ro)
    floor = roundoff_floor(oc, Uh, dt, cells=cells, trials=1)
    tol = np.maximum(RHS_TOL, 2.0 * floor)
    print(f"[parity] full size {cfgname}: rel err {np.array2string(err, precision=2)} "
          f"round-off floor {np.array2string(floor, precision=2)}", flush=True)
    for m in range(sc.ncomp):
        if err[m] > tol[m]:
            d = np.abs(Rg[m] - Ro[m])
            for w in np.argsort(d)[-5:]:
                c = int(cells[w])
                print(f"  comp {m} cell {c} (i={c % sc.nx}, j={(c // sc.nx) % sc.ny}, k={c // (sc.nx * sc.ny)}) "
                      f"gpu={Rg[m, w]:.17e} oracle={Ro[m, w]:.17e}", flush=True)
    assert np.all(err <= tol), (err, floor)
    if U1h is not None:
        ref1 = Uh.reshape(sc.ncomp, -1)[:, cells] + dt * Ro
        err1 = comp_rel(U1h[:, cells], ref1)
        assert np.all(err1 <= 1e-14), err1


DEGENERATE = [
    # (nx, ny, nz, bc per axis): single cells, lines and planes, exact and ragged tiles,
    # several z chunks, every boundary kind on small axes
    ((1, 1, 1), (WL.PERIODIC, WL.PERIODIC, WL.PERIODIC)),
    ((2, 3, 1), (WL.PERIODIC, WL.ZERO_GRADIENT, WL.PERIODIC)),
    ((1, 1, 7), (WL.ZERO_GRADIENT, WL.PERIODIC, WL.SYMMETRY)),
    ((3, 3, 3), (WL.SYMMETRY, WL.SYMMETRY, WL.SYMMETRY)),
    ((1, 19, 1), (WL.PERIODIC, WL.SYMMETRY, WL.ZERO_GRADIENT)),
    ((16, 16, 16), (WL.PERIODIC, WL.PERIODIC, WL.PERIODIC)),
    ((17, 16, 37), (WL.ZERO_GRADIENT, WL.PERIODIC, WL.SYMMETRY)),
]
DEGENERATE_VARIANTS = {
    "weno": {}, "char_teno": dict(scheme=1, recon=1),
}


DEGENERATE_MODELS = [(WL.EULER, "weno"), (WL.EULER, "char_teno"), (WL.NS, "weno"), (WL.NS, "char_teno"),
                     (WL.NS, "visc6"), (WL.DIM, "weno"), (WL.DIM, "char_teno")]
DEGENERATE_VARIANTS["visc6"] = dict(visc_order=6)


@pytest.mark.parametrize("model,variant", DEGENERATE_MODELS)
@pytest.mark.parametrize("shape,bcs", DEGENERATE)
def test_degenerate_grids_parity(shape, bcs, model, variant):
    """Grids of one cell, lines, planes, exact and ragged tiles and several z chunks:
    the tile masks, the halo mapping on axes shorter than the halo and the z-chunk
    seams against the oracle."""
    bc = tuple(b for b in bcs for _ in range(2))
    extra = dict(mu=0.02) if model == WL.NS else (dict(gamma1=1.66) if model == WL.DIM else {})
    case = WL.smooth_random(*shape, model=model, seed=41, bc=bc, **extra)
    kw = dict(DEGENERATE_VARIANTS[variant])
    if model == WL.DIM and variant != "weno":
        kw["thinc"] = 1    # characteristic TENO6-A with THINC
    oc = oracle_cfg(case, **kw)
    U = O.prim_to_cons(oc, case.W)
    dt = 0.3 * O.compute_dt(oc, U, 1.0)
    print(f"[parity] degenerate {shape} {bcs} model={model} {variant}", flush=True)
    Ro = O.rhs(oc, U, dt=dt)
    sc = solver_cfg(case, **kw)
    Rd = torch.empty_like(dev(U))
    S.rhs(sc, dev(U), Rd, dt=dt)
    err = comp_rel(host(Rd), Ro)
    floor = roundoff_floor(oc, U, dt)
    scale = np.abs(Ro).reshape(Ro.shape[0], -1).max(axis=1)
    # components that vanish identically (e.g. a velocity on a single-cell axis) compare absolutely
    absdiff = np.abs(host(Rd) - Ro).reshape(Ro.shape[0], -1).max(axis=1)
    ok = np.where(scale > 0, err <= np.maximum(RHS_TOL, 2.0 * floor), absdiff <= 1e-13)
    assert np.all(ok), (err, floor, absdiff)
