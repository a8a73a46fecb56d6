"""Host-side parts of the serving path (no GPU): the arena allocator, the
seeded request stream, and the argument checks of the batch entry points."""
import ctypes
import math

import numpy as np
import pytest

from paper_2402_05193_amd import workloads as WL

SV = pytest.importorskip("paper_2402_05193_amd.serving")
S = pytest.importorskip("paper_2402_05193_amd.solver")


def test_first_fit_alloc_release_coalesce():
    h = SV.FirstFit(10 * 256)
    a = h.alloc(300)   # 512 bytes
    b = h.alloc(256)
    c = h.alloc(1)
    assert (a, b, c) == (0, 512, 768)
    assert h.available == 10 * 256 - 1024
    assert h.alloc(4096) is None
    h.release(b, 256)
    assert h.alloc(512) == 1024          # the 256-byte hole is too small: first fit goes past it
    h.release(a, 300)
    h.release(c, 1)
    assert h.alloc(1024) == 0            # a, b, c coalesced into one range
    with pytest.raises(ValueError):
        h.release(0, 256)
        h.release(0, 256)


def test_first_fit_random_sequence_never_overlaps():
    rng = np.random.default_rng(5)
    h = SV.FirstFit(1 << 16)
    live = {}
    for _ in range(2000):
        if live and rng.random() < 0.45:
            off = rng.choice(list(live))
            h.release(off, live.pop(off))
        else:
            n = int(rng.integers(1, 4000))
            off = h.alloc(n)
            if off is not None:
                live[off] = n
        spans = sorted((o, o + SV._align(n)) for o, n in live.items())
        for (a0, a1), (b0, b1) in zip(spans, spans[1:]):
            assert a1 <= b0
        assert h.available + sum(SV._align(n) for n in live.values()) == h.size


def test_riemann_requests_are_seeded_and_in_range():
    a = [WL.riemann_request(i) for i in range(300)]
    b = [WL.riemann_request(i) for i in range(300)]
    assert a == b
    grids = set()
    for r in a:
        grids.add((r.nx, r.ny, r.nz))
        rl, ul, pl, gl = r.left
        rr, ur, pr, gr = r.right
        assert 0.1 <= rl <= 10 and 0.1 <= rr <= 10 and 0.1 <= pl <= 10 and 0.1 <= pr <= 10
        assert -1 <= ul <= 1 and -1 <= ur <= 1
        # no vacuum is generated (pressure positivity condition of the exact solution)
        assert 2 * math.sqrt(gl * pl / rl) / (gl - 1) + 2 * math.sqrt(gr * pr / rr) / (gr - 1) > ur - ul
        assert len(r.riemann_params()) == 2 + 2 * (7 if r.model == WL.DIM else 5)
        if r.model == WL.DIM:
            assert r.WL[6] == 1 - WL.ALPHA_EPS and r.WR[6] == WL.ALPHA_EPS
    assert grids == set(WL.SERVING_GRIDS)
    frac = np.mean([r.model == WL.DIM for r in a])
    assert 0.4 < frac < 0.6


def test_poisson_arrivals_rate():
    t = WL.poisson_arrivals(20000, 200.0)
    assert np.all(np.diff(t) > 0)
    gaps = np.diff(np.concatenate([[0.0], t]))
    assert abs(gaps.mean() - 1 / 200.0) < 0.03 / 200.0
    assert abs(gaps.std() / gaps.mean() - 1.0) < 0.03   # exponential gaps


def test_batch_entry_points_validate_arguments():
    L = S.lib()
    out = ctypes.c_size_t(0)
    assert L.batch_table_bytes(0, ctypes.byref(out)) == S.EINVAL
    assert L.batch_table_bytes(4, None) == S.ENULL
    assert L.batch_table_bytes(4, ctypes.byref(out)) == S.OK and out.value > 0
    h = ctypes.c_void_p(0)
    assert L.batch_create(4, ctypes.c_void_p(256), out.value, None) == S.ENULL
    assert L.batch_create(4, None, out.value, ctypes.byref(h)) == S.ENULL
    assert L.batch_create(4, ctypes.c_void_p(272), out.value, ctypes.byref(h)) == S.EALIGN
    assert L.batch_create(4, ctypes.c_void_p(512), 16, ctypes.byref(h)) == S.EINVAL
    assert L.batch_set(None, 0, None, None, None, None, None) == S.ENULL
    assert L.batch_step(None, 1, None) == S.ENULL
    assert L.batch_step_graph(None, 1, None) == S.ENULL
    assert L.batch_destroy(None) == S.OK
