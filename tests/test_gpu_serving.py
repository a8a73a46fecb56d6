"""Batched stepping of independent problems and the continuous-batching server.

Bars: a member's state after n batched steps is bitwise the state that
advance() gives for the same problem alone (the batched launch gives each
problem the same arithmetic); graph replays equal the eager batched steps
bitwise; FP64 members follow the FP64 oracle within the multi-step bar 1e-10;
FP32 members state their error against the FP64 oracle.
"""
import dataclasses
import math

import numpy as np
import pytest
import torch

import oracle as O
from paper_2402_05193_amd import serving as SV
from paper_2402_05193_amd import solver as S
from paper_2402_05193_amd import workloads as WL

pytestmark = pytest.mark.gpu

SMALL_GRIDS = ((24, 16, 16), (20, 12, 12), (32, 8, 8), (16, 8, 8))


def job(index, dtype, grid=None, steps=8, two_phase=None):
    grids = (grid,) if grid else SMALL_GRIDS
    frac = 0.5 if two_phase is None else (1.0 if two_phase else 0.0)
    req = WL.riemann_request(index, grids=grids, steps=steps, two_phase_fraction=frac)
    return SV.job_from_request(req, 0.0, dtype=dtype)


def tgv_job(index, n=16, steps=8):
    case = WL.taylor_green(n, viscous=True, with_field=False)
    cfg = S.config_from_case(case, dtype=S.F64, cfl=0.5)
    return SV.Job(index=index, cfg=cfg, case_id=S.CASE_TGV, params=[0.1, 1.0, 1e-3], steps=steps, arrival=0.0,
                  seed=2402)


def mixed_jobs(steps=8):
    return [job(0, S.F32, SMALL_GRIDS[0], steps, two_phase=False),
            job(1, S.F32, SMALL_GRIDS[1], steps, two_phase=True),
            job(2, S.F64, SMALL_GRIDS[2], steps, two_phase=False),
            tgv_job(3, steps=steps),
            job(4, S.F64, SMALL_GRIDS[3], steps, two_phase=True)]


def grouped_jobs(steps=8):
    """Members that share (model, precision, limiter) groups: batched launches of
    several problems (a group of one member runs the single-problem kernel)."""
    return [job(0, S.F32, SMALL_GRIDS[0], steps, two_phase=False),
            job(1, S.F32, SMALL_GRIDS[1], steps, two_phase=False),
            job(2, S.F32, SMALL_GRIDS[2], steps, two_phase=True),
            job(3, S.F32, SMALL_GRIDS[3], steps, two_phase=True),
            tgv_job(4, steps=steps),
            job(5, S.F64, SMALL_GRIDS[2], steps, two_phase=False)]


def option_jobs(steps=6):
    """Members with the reconstruction, interface and viscosity options, two per group
    (so that batched launches, not the single-problem path, run them) plus one alone:
    characteristic WENO5-Z (Euler FP64), TENO6-A (five-equation FP32), characteristic
    TENO6-A with THINC (five-equation FP64), THINC (five-equation FP32), Sutherland's
    viscosity law (NS FP64) and TENO6-A alone (NS FP64)."""
    out = []

    def add(j, **over):
        j.cfg = dataclasses.replace(j.cfg, **over)
        j.index = len(out)
        out.append(j)

    for g in SMALL_GRIDS[:2]:
        add(job(0, S.F64, g, steps, two_phase=False), recon=1)
    for g in SMALL_GRIDS[2:]:
        add(job(0, S.F32, g, steps, two_phase=True), scheme=1)
    for g in SMALL_GRIDS[:2]:
        add(job(0, S.F64, g, steps, two_phase=True), recon=1, scheme=1, thinc=1)
    for g in SMALL_GRIDS[1:3]:
        add(job(0, S.F32, g, steps, two_phase=True), thinc=1)
    for n in (16, 12):
        add(tgv_job(0, n=n, steps=steps), visc_law=2, T_ref=1.0, sutherland=0.4, gas_R=1.0)
    add(tgv_job(0, n=12, steps=steps), scheme=1)
    return out


def allocate(j):
    j.U = S.empty_state(j.cfg)
    j.ws = S.workspace(j.cfg)
    S.init_state(j.cfg, j.case_id, j.params, j.U, seed=j.seed)


def alone(j, nsteps):
    U = S.empty_state(j.cfg)
    ws = S.workspace(j.cfg)
    S.init_state(j.cfg, j.case_id, j.params, U, seed=j.seed)
    S.advance(j.cfg, U, nsteps, 0.0, ws)
    torch.cuda.synchronize()
    return U


def assert_bitwise(a, b, what):
    assert a.dtype == b.dtype and a.shape == b.shape
    same = torch.equal(a, b)
    if not same:
        d = (a.double() - b.double()).abs().max().item()
        raise AssertionError(f"{what}: not bitwise equal (max abs diff {d:.3e})")


def test_batch_members_join_and_leave_bitwise_alone():
    """Members join at different steps and leave after their own last step;
    each ends bitwise equal to its solo run."""
    jobs = mixed_jobs(steps=8)
    join_at = {0: 0, 2: 0, 1: 3, 3: 3, 4: 5}
    b = S.Batch(8)
    stream = torch.cuda.current_stream()
    active, done, step = [], [], 0
    while len(done) < len(jobs):
        fresh = []
        for j in jobs:
            if join_at[j.index] == step:
                allocate(j)
                fresh.append(j.index)
                active.append(j)
        if fresh or step == 0:
            b.set([(j.cfg, j.U, j.ws) for j in active], fresh=[j.index in fresh for j in active], stream=stream)
        b.step(1, stream=stream)
        step += 1
        left = []
        for j in active:
            j.steps_done += 1
            if j.steps_done == j.steps:
                done.append(j)
                left.append(j)
        if left:
            active = [j for j in active if j not in left]
            b.set([(j.cfg, j.U, j.ws) for j in active], stream=stream)
    torch.cuda.synchronize()
    for j in jobs:
        assert_bitwise(j.U, alone(j, j.steps), f"member {j.index} (model {j.cfg.model}, dtype {j.cfg.dtype})")
        # simulated time agrees with the solo run's
        ws = S.workspace(j.cfg)
        U = S.empty_state(j.cfg)
        S.init_state(j.cfg, j.case_id, j.params, U, seed=j.seed)
        t = S.advance(j.cfg, U, j.steps, 0.0, ws, t=0.0)
        assert S.workspace_time(j.cfg, j.ws) == t
    b.close()


def test_batch_members_with_options_bitwise_alone():
    """Members with the f3/f4 options (reconstruction family, THINC, a viscosity law)
    in one batch, stepped eagerly and through graph replays: every member ends bitwise
    equal to its solo run."""
    eager, graph = option_jobs(), option_jobs()
    for j in eager + graph:
        allocate(j)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        be, bg = S.Batch(16), S.Batch(16)
        be.set([(j.cfg, j.U, j.ws) for j in eager], fresh=[True] * len(eager), stream=stream)
        bg.set([(j.cfg, j.U, j.ws) for j in graph], fresh=[True] * len(graph), stream=stream)
        steps = eager[0].steps
        be.step(steps, stream=stream)
        for _ in range(steps):
            bg.step_graph(1, stream=stream)
        stream.synchronize()
        for je, jg in zip(eager, graph):
            what = (f"member {je.index} (model {je.cfg.model}, dtype {je.cfg.dtype}, recon {je.cfg.recon}, "
                    f"scheme {je.cfg.scheme}, thinc {je.cfg.thinc}, visc_law {je.cfg.visc_law})")
            print(f"[serving] {what}", flush=True)
            ref = alone(je, steps)
            assert torch.isfinite(ref).all()
            assert_bitwise(je.U, ref, what + " eager")
            assert_bitwise(jg.U, ref, what + " graph")
        be.close()
        bg.close()


def test_batch_graph_replays_equal_eager_steps():
    """The captured graph, replayed several times with eager work and
    synchronisations between the replays, matches the eager batched steps
    after every replay."""
    eager = grouped_jobs()
    graph = grouped_jobs()
    for j in eager + graph:
        allocate(j)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        be, bg = S.Batch(8), S.Batch(8)
        be.set([(j.cfg, j.U, j.ws) for j in eager], fresh=[True] * len(eager), stream=stream)
        bg.set([(j.cfg, j.U, j.ws) for j in graph], fresh=[True] * len(graph), stream=stream)
        scratch = torch.zeros(1 << 20, device="cuda")
        for rep in range(4):
            be.step(2, stream=stream)
            bg.step_graph(2, stream=stream)
            scratch.add_(1.0)  # unrelated eager work between replays
            stream.synchronize()
            for a, g in zip(eager, graph):
                assert_bitwise(g.U, a.U, f"replay {rep}, member {a.index}")
        assert float(scratch[0]) == 4.0
        be.close()
        bg.close()


def test_batch_graphs_survive_membership_changes():
    """Members join and leave at different steps; one batch steps through graph
    replays, another eagerly.  The graphs read the membership from the table, so
    they are reused across batch_set calls (fewer graphs than memberships), and
    every member ends bitwise equal in both batches (and to its solo run)."""
    eager = grouped_jobs(steps=8)
    graph = grouped_jobs(steps=8)
    join_at = {0: 0, 2: 0, 5: 0, 1: 3, 3: 3, 4: 5}
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        be, bg = S.Batch(8), S.Batch(8)
        active = {"e": [], "g": []}
        done, step, sets = 0, 0, 0
        while done < len(eager):
            changed = step == 0
            fresh = set()
            for je, jg in zip(eager, graph):
                if join_at[je.index] == step:
                    allocate(je)
                    allocate(jg)
                    active["e"].append(je)
                    active["g"].append(jg)
                    fresh.add(je.index)
                    changed = True
            if changed:
                for key, b in (("e", be), ("g", bg)):
                    b.set([(j.cfg, j.U, j.ws) for j in active[key]], fresh=[j.index in fresh for j in active[key]],
                          stream=stream)
                sets += 1
            be.step(1, stream=stream)
            bg.step_graph(1, stream=stream)
            step += 1
            for key in ("e", "g"):
                for j in active[key]:
                    j.steps_done += 1
            left = [j for j in active["e"] if j.steps_done == j.steps]
            if left:
                done += len(left)
                for key, b in (("e", be), ("g", bg)):
                    active[key] = [j for j in active[key] if j.steps_done < j.steps]
                    b.set([(j.cfg, j.U, j.ws) for j in active[key]], stream=stream)
                sets += 1
        stream.synchronize()
        print(f"[serving] {sets} memberships, {bg.graph_count()} graphs captured", flush=True)
        assert 1 <= bg.graph_count() < sets
        for je, jg in zip(eager, graph):
            assert_bitwise(jg.U, je.U, f"member {je.index} graph vs eager")
            assert_bitwise(jg.U, alone(jg, jg.steps), f"member {jg.index} graph vs alone")
        be.close()
        bg.close()


def test_batched_fp64_members_follow_the_oracle():
    """FP64 members of a mixed batch against the oracle's CFL-mode advance."""
    jobs = mixed_jobs(steps=8)
    for j in jobs:
        allocate(j)
    b = S.Batch(8)
    b.set([(j.cfg, j.U, j.ws) for j in jobs], fresh=[True] * len(jobs))
    b.step(8)
    torch.cuda.synchronize()
    for j in jobs:
        oc = O.Config(**{k: getattr(j.cfg, k) for k in ("nx", "ny", "nz", "dx", "dy", "dz", "model", "bc", "gamma1",
                                                       "pinf1", "gamma2", "pinf2", "mu", "prandtl", "positivity")})
        U0 = S.empty_state(S.Config(**{**j.cfg.__dict__, "dtype": S.F64}))
        S.init_state(S.Config(**{**j.cfg.__dict__, "dtype": S.F64}), j.case_id, j.params, U0, seed=j.seed)
        torch.cuda.synchronize()
        Uo, _ = O.advance(oc, U0.cpu().numpy(), 8, 0.0, cfl=0.5)
        g = j.U.double().cpu().numpy()
        nc = Uo.shape[0]
        rel = max(np.abs(g[m] - Uo[m]).max() / max(np.abs(Uo[m]).max(), 1e-300) for m in range(nc))
        v0 = 2 if nc == 7 else 1
        mom = np.abs(Uo[v0:v0 + 3]).max()
        rel_m = max(np.abs(g[m] - Uo[m]).max() / mom for m in range(v0, v0 + 3))
        l1 = np.abs(g - Uo).sum() / np.abs(Uo).sum()
        print(f"member {j.index} model {j.cfg.model} dtype {j.cfg.dtype}: max rel {rel:.3e}, momentum {rel_m:.3e},"
              f" L1 rel {l1:.3e}", flush=True)
        if j.cfg.dtype == S.F64:
            scalar = [m for m in range(nc) if not v0 <= m < v0 + 3]
            worst = max(max(np.abs(g[m] - Uo[m]).max() / max(np.abs(Uo[m]).max(), 1e-300) for m in scalar), rel_m)
            assert worst <= 1e-10, (j.index, worst)
        else:
            # FP32 against the FP64 oracle (stated error, L1 relative): smooth-ish single-phase
            # fields stay near FP32 round-off; the two-phase member carries 1e-8 volume
            # fractions through an interface and a shock (FP32 tolerances are 100x the FP64 ones)
            assert l1 <= (1e-5 if j.cfg.model == S.EULER else 5e-3), (j.index, l1)
    b.close()


@pytest.mark.parametrize("use_graph,fill,policy", [(False, None, "fcfs"), (True, None, "fcfs"), (True, 40, "fcfs"),
                                                   (True, 40, "srpt"), (False, None, "srpt"), (True, 40, "srpt-oldest")])
def test_server_results_same_alone_and_in_the_mix(use_graph, fill, policy):
    """Continuous batching with admission by memory (and by GPU fill), in arrival
    order or least remaining work first (members paused between steps): an arena
    that holds only a few requests, requests arriving while others run; every
    result equals the request's solo result bitwise, and so does the
    one-at-a-time path's."""
    jobs = [job(i, S.F32 if i % 3 else S.F64, steps=6 + i % 3) for i in range(9)]
    for k, j in enumerate(jobs):
        j.arrival = 0.002 * k
    biggest = max(SV.Server.job_bytes(j.cfg) for j in jobs)
    srv = SV.Server(pool_bytes=3 * biggest, max_batch=4, use_graph=use_graph, fill_workgroups=fill,
                    policy=policy.split("-")[0], protect_oldest=policy.endswith("oldest"))
    st = srv.run_batched(jobs, keep_results=True)
    assert st.n == len(jobs) and st.max_batch_seen <= 4
    assert all(j.finish >= j.arrival for j in jobs)
    seq = [SV.Job(**{**j.__dict__, "U": None, "ws": None, "result": None, "finish": None, "steps_done": 0})
           for j in jobs]
    st2 = srv.run_sequential(seq, keep_results=True)
    torch.cuda.synchronize()
    for j, q in zip(jobs, seq):
        ref = alone(j, j.steps)
        assert_bitwise(j.result, ref, f"batched request {j.index}")
        assert_bitwise(q.result, ref, f"sequential request {j.index}")
    assert srv.heap.available == srv.heap.size
    print("batched", st.summary(), "\nsequential", st2.summary(), flush=True)
    srv.close()
