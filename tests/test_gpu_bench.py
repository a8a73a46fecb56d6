"""The benchmark's JSON line on a small grid: the keys it must carry and the
arithmetic that ties its figures together (throughput from the timed region,
the roofline fraction from the algorithmic FLOPs per cell)."""
import json
import sys

import pytest

pytestmark = pytest.mark.gpu

KEYS = ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
        "scaling", "vs_baseline", "dtype", "data", "config", "roofline")


def _run(monkeypatch, capsys, *extra):
    import bench
    monkeypatch.setattr(sys, "argv", ["bench.py", "--steps", "3", "--warmup", "1", "--serve-requests", "0",
                                      "--no-adjoint", *extra])
    bench.main()
    lines = [l for l in capsys.readouterr().out.splitlines() if l.startswith("{")]
    assert lines, "no JSON line printed"
    return bench, json.loads(lines[-1])


@pytest.mark.parametrize("extra", [("--n", "64"), ("--n", "48", "--model", "euler", "--dtype", "f32"),
                                   ("--n", "64", "--model", "dim")])
def test_json_line_contract(monkeypatch, capsys, extra):
    bench, d = _run(monkeypatch, capsys, "--no-cpu-baseline", *extra)
    for k in KEYS:
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 3 and d["warmup"] == 1
    assert d["higher_is_better"] is True and d["vs_baseline"] is None
    assert d["unit"] == "cell-updates/s" and d["state_finite"] is True
    assert isinstance(d["config"]["workload"], str) and d["config"]["workload"]
    cells = d["config"]["cells"]
    # value: three stage updates of every cell per step over the whole timed region
    assert d["value"] == pytest.approx(cells * 3 / (d["ms_per_step"] * 1e-3), rel=1e-9)
    r = d["roofline"]
    assert r["bound"] == "alu" and r["unit"] == "TFLOP/s"
    assert r["peak"] == 78.6      # FP64 vector; FP32 without packed operations issues at the same rate
    assert r["achieved"] == pytest.approx(r["flops_per_cell"] * cells / (d["stage_ms"]["mean"] * 1e-3) / 1e12,
                                          rel=1e-9)
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], rel=1e-12)
    assert 0.0 < r["frac"] < 1.0
    # no traffic record exists for these small grids
    assert r["traffic"] is None
    assert "cpu_baseline" not in d


def test_cpu_baseline_object(monkeypatch, capsys):
    _, d = _run(monkeypatch, capsys, "--n", "32")
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["unit"] == "cell-updates/s"
    assert c["value"] > 0 and c["cores"] >= 1 and "32x32x32" in c["sample"]
