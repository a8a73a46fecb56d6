"""Calibration of the parity bar's round-off floor, CPU only.

The low-Mach Taylor-Green vortex (1/(gamma Ma^2) ~ 71 in the pressure flux)
loses digits in the flux difference, so R is ill-conditioned: two correct FP64
evaluations that round differently disagree by more than 1e-12 relative.  The
GPU parity tests take the bar as max(1e-12, 2 x floor), with the floor measured
by moving every input by one unit in the last place.  This test measures the
floor independently, as the difference between the oracle built with
multiply-add contraction off (the reference build) and on (the same source,
fused wherever the compiler can), and checks that the two estimates agree
within a factor of three and that both exceed 1e-12 on density and energy at
C1 (32^3, Euler).
"""
import os
import subprocess
import sys
import tempfile

import numpy as np

import oracle as O
from paper_2402_05193_amd import workloads as WL

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def comp_rel(g, r):
    nc = r.shape[0]
    g = g.reshape(nc, -1)
    r = r.reshape(nc, -1)
    mom = np.abs(r[1:4]).max()
    return np.array([np.abs(g[m] - r[m]).max() / (mom if 1 <= m < 4 else np.abs(r[m]).max()) for m in range(nc)])


CHILD = """
import sys, numpy as np
sys.path.insert(0, {root!r})
import oracle as O
O._LIB_PATH = {lib!r}
from paper_2402_05193_amd import workloads as WL
case = WL.taylor_green(32)
oc = O.Config(**case.cfg_kwargs())
np.save({out!r}, O.rhs(oc, O.prim_to_cons(oc, case.W), dt=1e-3))
"""


def test_contraction_floor_matches_ulp_floor_at_c1():
    case = WL.taylor_green(32)
    oc = O.Config(**case.cfg_kwargs())
    U = O.prim_to_cons(oc, case.W)
    R = O.rhs(oc, U, dt=1e-3)
    rng = np.random.default_rng(1)
    ulp = np.zeros(5)
    for _ in range(2):
        Up = U * (1.0 + rng.choice([-1.0, 1.0], size=U.shape) * 2.0 ** -53)
        ulp = np.maximum(ulp, comp_rel(O.rhs(oc, Up, dt=1e-3), R))
    with tempfile.TemporaryDirectory() as tmp:
        lib = os.path.join(tmp, "liboracle_fma.so")
        out = os.path.join(tmp, "R.npy")
        subprocess.run(["make", "-s", "-C", os.path.join(ROOT, "oracle"), "-B", "fma", f"FMA_OUT={lib}"], check=True)
        subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT, lib=lib, out=out)], check=True)
        Rf = np.load(out)
    fma = comp_rel(Rf, R)
    print("ulp floor", ulp, "contraction floor", fma)
    assert not np.array_equal(Rf, R)             # the contracted build did round differently
    for m in (0, 4):
        assert fma[m] > 1e-12 and ulp[m] > 1e-12
    assert np.all(fma <= 3.0 * ulp) and np.all(ulp <= 3.0 * fma)
