"""GPU parity of the positivity limiters (Sec. 3.3) while they act, with the
decisions of every face compared (through the C ABI's rhs_flags).

Decision masks: bit 0 / bit 1 = the interpolation limiter replaced the left /
right reconstructed state by its cell state, bit 2 = the flux limiter switched
to the first-order HLLC flux.  GPU and oracle take each decision from their own
floating-point evaluation of the same input, so a face whose admissibility
margin is at the rounding level may decide differently.  The tests compare the
masks bit for bit and accept a differing face only if it is such a tie: the
oracle's own decision at that face changes when the input moves by one unit in
the last place.  Every flip is printed with its face and both decisions.  R is
compared at the round-off floor on the cells away from flipped faces.

Cases: the interpolation limiter forced everywhere; the flux limiter alone at
the closed-form thresholds of the oracle pins (tests/test_oracle_limiters.py)
and at a large time step on three-dimensional fields; the five-equation
shock-bubble (64 x 32 x 32) along 150 CFL steps through shock-bubble contact,
every stage input of every fifth step from step 35 (the oracle's own
trajectory, so both sides see the same input); the same states with THINC and
characteristic TENO6-A; and the full-size 256 x 128 x 128 shock-bubble advanced
on the GPU past contact until the limiters act, in the benchmark's launch
configuration, on sampled cells next to limited faces.
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2402_05193_amd import solver as S
from paper_2402_05193_amd import workloads as WL
from test_gpu_parity import comp_rel, dev, host, oracle_cfg, roundoff_floor, solver_cfg
from test_oracle_limiters import between_thresholds, faces_flux, single_phase_case, trip_lambda

pytestmark = pytest.mark.gpu

DIRS = "xyz"


def gpu_flags(sc, U, dt, ws=None):
    Ud = dev(U)
    R, views = S.rhs_flags(sc, Ud, torch.empty_like(Ud), dt=dt, ws=ws)
    torch.cuda.synchronize()
    return host(R), [v.cpu().numpy() for v in views]


def perturbed_flags(oc, U, dt, trials=3, seed=3):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(trials):
        Up = U * (1.0 + rng.choice([-1.0, 1.0], size=U.shape) * 2.0 ** -52)
        out.append(O.rhs(oc, Up, dt=dt, return_flags=True)[1])
    return out


def compare_masks(oc, U, dt, fg, fo, label):
    """Bitwise comparison of the decision masks; returns (number of decisions set on
    either side, number of flipped faces, boolean mask of cells next to a flip)."""
    ncell_mask = np.zeros((oc.nz, oc.ny, oc.nx), dtype=bool)
    flips = []
    for d in range(3):
        diff = np.argwhere(fg[d] != fo[d])
        for k, j, i in diff:
            flips.append((d, int(k), int(j), int(i), int(fg[d][k, j, i]), int(fo[d][k, j, i])))
    if flips:
        pert = perturbed_flags(oc, U, dt)
        for d, k, j, i, g, o in flips:
            tie = any(int(p[d][k, j, i]) != o for p in pert)
            print(f"  [{label}] flip {DIRS[d]} face (k={k}, j={j}, i={i}): gpu {g:03b} oracle {o:03b} "
                  f"{'(oracle decision moves with a 1-ulp input change)' if tie else '(NOT a tie)'}", flush=True)
            assert tie, (label, d, k, j, i, g, o)
            # the two cells that share the face: the one at the face index along d and
            # the one before it
            idx = [k, j, i]
            if idx[2 - d] < (oc.nx, oc.ny, oc.nz)[d]:
                ncell_mask[tuple(idx)] = True
            idx[2 - d] -= 1
            if idx[2 - d] >= 0:
                ncell_mask[tuple(idx)] = True
    nset = sum(int(((a != 0) | (b != 0)).sum()) for a, b in zip(fg, fo))
    return nset, len(flips), ncell_mask


def compare_rhs(oc, U, dt, Rg, Ro, skip, label, floor=None):
    nc = oc.ncomp
    keep = ~skip.reshape(-1)
    g = Rg.reshape(nc, -1)[:, keep]
    r = Ro.reshape(nc, -1)[:, keep]
    err = comp_rel(g, r)
    if floor is None:
        floor = roundoff_floor(oc, U, dt, trials=1)
    tol = np.maximum(1e-12, 2.0 * floor)
    print(f"  [{label}] R rel err {np.array2string(err, precision=2)} floor {np.array2string(floor, precision=2)} "
          f"({int(skip.sum())} cells next to flips left out)", flush=True)
    assert np.all(err <= tol), (label, err, floor)


def check_case(oc, sc, U, dt, label, floor=None):
    Ro, fo = O.rhs(oc, U, dt=dt, return_flags=True)
    Rg, fg = gpu_flags(sc, U, dt)
    nset, nflip, skip = compare_masks(oc, U, dt, fg, fo, label)
    compare_rhs(oc, U, dt, Rg, Ro, skip, label, floor)
    bits = [int(sum(((f >> b) & 1).sum() for f in fo)) for b in range(3)]
    print(f"  [{label}] decisions (oracle): IL left {bits[0]}, IL right {bits[1]}, FL {bits[2]}; "
          f"faces with a decision {nset}, flips {nflip}", flush=True)
    return bits, nflip


def test_rhs_flags_returns_the_rhs():
    case = WL.shock_bubble(48, 24, 24)
    oc = oracle_cfg(case)
    sc = solver_cfg(case)
    U = dev(O.prim_to_cons(oc, case.W))
    R1 = S.rhs(sc, U, torch.empty_like(U), dt=2e-7)
    R2, views = S.rhs_flags(sc, U, torch.empty_like(U), dt=2e-7)
    assert torch.equal(R1, R2)
    assert [tuple(v.shape) for v in views] == [(24, 24, 49), (24, 25, 48), (25, 24, 48)]
    # limiters off: every byte 0 and R as rhs computes it
    sc0 = solver_cfg(case, positivity=0)
    flags = torch.full((S.limiter_flag_bytes(sc0),), 7, dtype=torch.uint8, device="cuda")
    R3, _ = S.rhs_flags(sc0, U, torch.empty_like(U), dt=2e-7, flags=flags)
    assert int(flags.max()) == 0
    assert torch.equal(R3, S.rhs(sc0, U, torch.empty_like(U), dt=2e-7))


@pytest.mark.parametrize("model", [WL.EULER, WL.DIM])
def test_forced_interpolation_limiter(model):
    """Tolerance far above every state: the interpolation limiter replaces both
    states of every face; the result is the first-order Godunov scheme."""
    extra = dict(gamma1=1.66) if model == WL.DIM else {}
    case = WL.smooth_random(19, 13, 11, model=model, seed=51, bc=(WL.PERIODIC, WL.PERIODIC, WL.ZERO_GRADIENT,
                                                                  WL.ZERO_GRADIENT, WL.SYMMETRY, WL.SYMMETRY),
                            **extra)
    oc = oracle_cfg(case, positivity=1, eps_rho=1e30)
    sc = solver_cfg(case, positivity=1, eps_rho=1e30)
    U = O.prim_to_cons(oc, case.W)
    dt = 0.3 * O.compute_dt(oc, U, 1.0)
    bits, nflip = check_case(oc, sc, U, dt, f"forced IL model {model}")
    nfaces = sum(O.face_counts(oc))
    assert bits[0] == nfaces and bits[1] == nfaces
    assert nflip == 0


@pytest.mark.parametrize("ny,nz", [(1, 1), (4, 3)])
def test_flux_limiter_at_closed_form_thresholds(ny, nz):
    """The oracle pin's advected density ramp: only the flux limiter acts, on the
    faces whose pseudo-time threshold lies below dt."""
    n = 40
    cfg, W = single_phase_case(n, ny, nz)
    D = 1 + (ny > 1) + (nz > 1)
    U = O.prim_to_cons(cfg, W)
    F0 = faces_flux(O.rhs(cfg, U, dt=1e-6), cfg.dx, W[0, 0, 0, 0], 0)
    lam = trip_lambda(W[0, 0, 0], F0) / (2.0 * D)
    sc = S.Config(nx=n, ny=ny, nz=nz, model=S.EULER, bc=cfg.bc, positivity=1, gamma1=1.4)
    for k, dt in between_thresholds(lam):
        bits, nflip = check_case(cfg, sc, U, dt, f"FL ramp D={D} k={k}")
        assert bits[2] == k * ny * nz and bits[0] == 0 and bits[1] == 0
        assert nflip == 0


@pytest.mark.parametrize("model", [WL.EULER, WL.DIM])
def test_flux_limiter_at_a_large_time_step(model):
    """Three-dimensional fields at eight times the CFL time step: the flux limiter
    trips on faces of every direction (the interpolation limiter stays off)."""
    extra = dict(gamma1=1.66) if model == WL.DIM else {}
    case = WL.smooth_random(21, 17, 15, model=model, seed=52, amplitude=0.45,
                            bc=(WL.ZERO_GRADIENT,) * 2 + (WL.PERIODIC,) * 2 + (WL.SYMMETRY,) * 2, **extra)
    oc = oracle_cfg(case, positivity=1)
    sc = solver_cfg(case, positivity=1)
    U = O.prim_to_cons(oc, case.W)
    dt = 8.0 * O.compute_dt(oc, U, 1.0)
    bits, nflip = check_case(oc, sc, U, dt, f"FL large dt model {model}")
    assert bits[2] > 0
    per_dir = [int(((f & 4) != 0).sum()) for f in O.rhs(oc, U, dt=dt, return_flags=True)[1]]
    assert all(c > 0 for c in per_dir), per_dir


@pytest.fixture(scope="module")
def sbi_trajectory():
    """The oracle's 64 x 32 x 32 shock-bubble: 150 CFL-0.5 steps, stage inputs kept
    for every fifth step from step 35 (the limiters first act near step 40)."""
    case = WL.shock_bubble(64, 32, 32)
    oc = oracle_cfg(case)
    U = O.prim_to_cons(oc, case.W)
    U0 = U.copy()
    kept = []
    t = 0.0
    print("[limiters] oracle shock-bubble 64x32x32, 150 steps ...", flush=True)
    for step in range(150):
        dt = O.compute_dt(oc, U, 0.5)
        U1 = O.rk3_stage(oc, 1, U, U, dt)
        U2 = O.rk3_stage(oc, 2, U, U1, dt)
        if step >= 35 and step % 5 == 0:
            kept.append((step, dt, U.copy(), U1, U2))
        U = O.rk3_stage(oc, 3, U, U2, dt)
        t += dt
    return case, oc, U0, U, t, kept


def test_shock_bubble_limiter_decisions_along_the_trajectory(sbi_trajectory):
    case, oc, _, _, _, kept = sbi_trajectory
    sc = solver_cfg(case)
    totals = np.zeros(3, dtype=np.int64)
    flips = 0
    for step, dt, *stages in kept:
        for s, Us in enumerate(stages):
            bits, nflip = check_case(oc, sc, Us, dt, f"sbi step {step} stage {s + 1}")
            totals += bits
            flips += nflip
    print(f"[limiters] shock-bubble trajectory: {len(kept) * 3} stage inputs, decisions IL left {totals[0]}, "
          f"IL right {totals[1]}, FL {totals[2]}; flipped faces {flips}", flush=True)
    assert totals[0] + totals[1] > 100 and totals[2] > 50


@pytest.mark.parametrize("variant", ["thinc", "char_teno_thinc"])
def test_shock_bubble_limiter_decisions_with_thinc(sbi_trajectory, variant):
    case, _, _, _, _, kept = sbi_trajectory
    kw = dict(thinc=1) if variant == "thinc" else dict(thinc=1, scheme=1, recon=1)
    oc = oracle_cfg(case, **kw)
    sc = solver_cfg(case, **kw)
    totals = np.zeros(3, dtype=np.int64)
    for step, dt, Un, _, _ in kept[::4]:
        bits, _ = check_case(oc, sc, Un, dt, f"sbi {variant} step {step}")
        totals += bits
    print(f"[limiters] shock-bubble {variant}: decisions {totals}", flush=True)
    assert totals.sum() > 0


def test_shock_bubble_150_steps(sbi_trajectory):
    """The GPU's own 150-step trajectory (CFL mode) against the oracle's: the
    spec bar of 1e-10 after 100 steps, per component relative to the
    component's maximum, and the simulated time."""
    case, oc, U0, Uo, to, _ = sbi_trajectory
    sc = solver_cfg(case, cfl=0.5)
    Ud = dev(U0)
    t = S.advance(sc, Ud, 150, 0.0, S.workspace(sc), t=0.0)
    err = comp_rel(host(Ud), Uo)
    print(f"[limiters] shock-bubble 150 steps: rel err {np.array2string(err, precision=2)}, "
          f"time {t:.9e} vs {to:.9e}", flush=True)
    assert t == pytest.approx(to, rel=1e-12)
    assert np.all(err <= 1e-10), err


@pytest.mark.parametrize("opt", ["", "char_teno_thinc"])
def test_full_size_post_contact_limiters(opt):
    """256 x 128 x 128 shock-bubble advanced on the GPU past shock-bubble contact
    (near step 55) until the limiters act, in the launch configuration the
    benchmark times: R and
    the six face decisions of sampled cells -- 200 random cells and up to 400
    cells next to limited faces -- against the oracle evaluated cell by cell on
    the GPU's state."""
    kw = dict(thinc=1, scheme=1, recon=1) if opt else {}
    case = WL.shock_bubble(256, 128, 128, with_field=False)
    sc = solver_cfg(case, cfl=0.5, **kw)
    rho2, u2, p2 = case.meta["post_shock"]
    H = case.meta["H"]
    params = [0.060, 0.090, H / 2, H / 2, 0.25 * H, WL.ALPHA_EPS, rho2, u2, p2, 1.2041, 101325.0, 0.1660]
    U = S.init_state(sc, S.CASE_SBI, params, S.empty_state(sc))
    ws = S.workspace(sc)
    dtd = torch.zeros(1, dtype=torch.float64, device="cuda")
    # advance in blocks of 50 CFL steps until the limiters act (after contact)
    steps = 0
    while True:
        S.advance(sc, U, 50, 0.0, ws)
        steps += 50
        S.compute_dt(sc, U, dtd, ws)
        dt = float(dtd.item())
        R, views = S.rhs_flags(sc, U, torch.empty_like(U), dt=dt)
        nlim = sum(int(torch.count_nonzero(v)) for v in views)
        print(f"[limiters] full size {opt or 'default'}: {steps} GPU steps, {nlim} limited faces", flush=True)
        if nlim > 0 or steps >= 400:
            break
    torch.cuda.synchronize()
    Uh = host(U)
    Rh = host(R).reshape(sc.ncomp, -1)
    fx, fy, fz = [v.cpu().numpy() for v in views]
    del R, U, ws
    torch.cuda.empty_cache()
    nx, ny, nz = sc.nx, sc.ny, sc.nz
    # cells with a limited face
    lim = np.zeros((nz, ny, nx), dtype=bool)
    lim |= fx[:, :, :-1] != 0
    lim |= fx[:, :, 1:] != 0
    lim |= fy[:, :-1, :] != 0
    lim |= fy[:, 1:, :] != 0
    lim |= fz[:-1] != 0
    lim |= fz[1:] != 0
    cand = np.flatnonzero(lim)
    print(f"[limiters] full size: {len(cand)} cells next to a limited face", flush=True)
    # the default configuration (primitive WENO5-Z, no THINC) at this resolution: no
    # limiter acts in 400 steps (nor with THINC alone); the sampled cells then check
    # that the oracle agrees
    if opt:
        assert len(cand) > 0
    rng = np.random.default_rng(11)
    cells = rng.integers(0, nx * ny * nz, 200)
    if len(cand):
        cells = np.concatenate([cells, rng.choice(cand, min(400, len(cand)), replace=False)])
    oc = oracle_cfg(case, **kw)
    Ro, fo = O.rhs_cells(oc, Uh, cells, dt=dt, return_flags=True)
    k, j, i = cells // (nx * ny), (cells // nx) % ny, cells % nx
    fg = np.stack([fx[k, j, i], fx[k, j, i + 1], fy[k, j, i], fy[k, j + 1, i], fz[k, j, i], fz[k + 1, j, i]], axis=1)
    bad = np.argwhere(fg != fo)
    skip = np.zeros(len(cells), dtype=bool)
    if len(bad):
        rngp = np.random.default_rng(5)
        pert = []
        for _ in range(3):
            Up = Uh * (1.0 + rngp.choice([-1.0, 1.0], size=Uh.shape) * 2.0 ** -52)
            pert.append(O.rhs_cells(oc, Up, cells, dt=dt, return_flags=True)[1])
        for c, f in bad:
            tie = any(int(p[c, f]) != int(fo[c, f]) for p in pert)
            print(f"  flip cell {int(cells[c])} face {['-x', '+x', '-y', '+y', '-z', '+z'][f]}: gpu {int(fg[c, f]):03b} "
                  f"oracle {int(fo[c, f]):03b} {'(tie)' if tie else '(NOT a tie)'}", flush=True)
            assert tie
            skip[c] = True
    bits = [int(((fo >> b) & 1).sum()) for b in range(3)]
    print(f"[limiters] full size: sampled face decisions IL left {bits[0]}, IL right {bits[1]}, FL {bits[2]}; "
          f"flips {len(bad)}", flush=True)
    assert (bits[0] + bits[1] + bits[2] > 0) == (len(cand) > 0)
    keep = ~skip
    err = comp_rel(Rh[:, cells][:, keep], Ro[:, keep])
    floor = roundoff_floor(oc, Uh, dt, cells=cells[keep], trials=1)
    tol = np.maximum(1e-12, 2.0 * floor)
    print(f"[limiters] full size: R rel err {np.array2string(err, precision=2)} floor "
          f"{np.array2string(floor, precision=2)}", flush=True)
    Rk, ck = Rh[:, cells][:, keep], cells[keep]
    for m in range(sc.ncomp):
        if err[m] > tol[m]:
            d = np.abs(Rk[m] - Ro[m, keep])
            for w in np.argsort(d)[-4:]:
                c = int(ck[w])
                a = Uh[6].reshape(-1)[c] if sc.ncomp == 7 else 0.0
                print(f"  comp {m} cell {c} (i={c % nx}, j={(c // nx) % ny}, k={c // (nx * ny)}) alpha1 {a:.6e} "
                      f"gpu={Rk[m, w]:.17e} oracle={Ro[m, keep][w]:.17e}", flush=True)
    assert np.all(err <= tol), (err, floor)
