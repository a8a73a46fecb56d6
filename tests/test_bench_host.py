"""Host-side pieces of the benchmark (CPU only): the FLOP count per cell that the
roofline uses, the traffic record lookup and the one-GPU rule."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_flops_per_cell_of_the_stage_variants():
    # NS with 4th-order viscous fluxes, Euler, five-equation model: 15 or 21 WENO5-Z pairs,
    # three HLLC faces, viscous faces, U -> W, divergence and the RK combination
    assert bench.flops_per_cell(1) == 2067
    assert bench.flops_per_cell(0) == 1781
    assert bench.flops_per_cell(2) == 2414
    # the variants cost more than the default
    assert bench.flops_per_cell(1, scheme=1) > bench.flops_per_cell(1, recon=1) > bench.flops_per_cell(1)
    assert bench.flops_per_cell(1, visc_order=6) > bench.flops_per_cell(1)


def test_bytes_per_cell():
    assert bench.bytes_per_cell(5, 8, 1) == 80
    assert bench.bytes_per_cell(5, 8, 2) == 120
    assert bench.bytes_per_cell(7, 4, 3) == 84


def test_traffic_record_needs_the_current_kernel(tmp_path, monkeypatch):
    (tmp_path / "p.md").write_text("traffic-record: kernel=abc workload=ns-f64-256 fetch_bytes=10 write_bytes=5\n")
    (tmp_path / "q.md").write_text("valu-record: kernel=xyz workload=dim-f64-256 insts_per_cell=7.5\n"
                                   "traffic-record: kernel=xyz workload=dim-f64-256 fetch_bytes=3 write_bytes=4\n")
    monkeypatch.setattr(bench, "PROFILES_DIR", str(tmp_path))
    # each workload's record is matched against its own stage kernel's fingerprint
    fps = {bench.WORKLOAD_KERNELS["ns-f64-256"]: "abc", bench.WORKLOAD_KERNELS["dim-f64-256"]: "xyz"}
    monkeypatch.setattr(bench, "stage_kernel_hash", lambda symbol=bench.STAGE_KERNEL_SYMBOL: fps[symbol])
    assert bench.measured_traffic("ns-f64-256") == 15
    assert bench.measured_traffic("dim-f64-256") == 7
    assert bench.measured_valu_insts_per_cell("dim-f64-256") == 7.5
    assert bench.measured_traffic("ns-f32-256") is None     # no kernel known for the workload
    fps[bench.WORKLOAD_KERNELS["ns-f64-256"]] = "def"       # the kernel changed since the record
    assert bench.measured_traffic("ns-f64-256") is None
    assert bench.measured_traffic("dim-f64-256") == 7


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode == 2
    assert json.loads(p.stdout.strip().splitlines()[-1])["n_gpus"] == 2
