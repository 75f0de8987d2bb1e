"""The benchmark's output contract, on a small vortex: one JSON line with the
metric, the whole-job value (the FP32 form's MLUPS), the roofline object of the
dominant kernel (achieved / peak = frac; traffic null unless the committed
counter summary was taken on this lattice size), the oracle's CPU baseline and
the per-form errors against FP64, in a separate process as the benchmark is
run."""
import json
import math
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_prints_one_json_line_with_roofline_and_cpu_baseline():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--n", "64", "--settle", "4", "--warmup", "2",
           "--steps", "5", "--closure-steps", "10", "--cpu-planes", "2", "--cpu-steps", "1"]
    print("bench:", " ".join(cmd[1:]), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.splitlines() if l.strip()]
    assert len(lines) == 1, r.stdout
    d = json.loads(lines[0])
    for k in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
              "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline"):
        assert k in d, k
    assert d["n_gpus"] == 1 and d["steps"] == 5 and d["warmup"] == 2
    assert d["unit"] == "MLUPS" and d["dtype"] == "f32" and d["higher_is_better"] is True
    assert d["vs_baseline"] is None
    assert "64^3" in d["config"]["workload"]
    f32 = d["forms"]["f32"]
    assert d["value"] == pytest.approx(f32["mlups"], rel=1e-3)
    # value and ms_per_step describe the same timing
    assert d["value"] == pytest.approx(64 ** 3 / (d["ms_per_step"] * 1e-3) / 1e6, rel=1e-3)
    roof = d["roofline"]
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    # algorithmic bytes: 27 reads + 27 writes of 4 bytes per node and step
    assert roof["achieved"] == pytest.approx(d["value"] * 1e6 * 216 / 1e9, rel=1e-3)
    assert roof["frac"] == pytest.approx(roof["achieved"] / roof["peak"], abs=1e-4)
    assert roof["traffic"] is None  # the counter summary covers the 512^3 lattice only
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["unit"] == "MLUPS" and cb["value"] > 0 and cb["cores"] >= 1
    for st in ("f64", "f32", "f16dev", "bf16dev"):
        form = d["forms"][st]
        assert form["mlups"] > 0 and math.isfinite(form["kinetic_energy_per_node"])
        assert abs(form["mass_rel_drift"]) < 1e-6
    assert d["forms"]["f64"]["ke_rel_err_vs_f64"] == 0.0
    assert d["forms"]["f32"]["ke_rel_err_vs_f64"] < 1e-6
    for g in ("channel_192x96x96", "channel_384x192x192"):
        cf = d["closure_forms"][g]
        assert cf["f32"]["vs_f32_plain"] == 1.0
        assert all(cf[k]["finite"] for k in cf if k != "steps")
    cr = d["copy_reference"]
    assert 1000 < cr["copy_GBs"] < 8000
    assert cr["f32_achieved_over_copy"] == pytest.approx(roof["achieved"] / cr["copy_GBs"], rel=1e-3)
    # cost of plain FP32 at the closure's mean-flow error over the closure form's
    cost = d["closure_forms"]["cost_at_equal_error"]
    r = cost["plain_refinement_for_equal_error"]
    assert r > 1.0 and cost["U_error_closure"] < cost["U_error_plain_f32"]
    mlups = d["closure_forms"]["channel_192x96x96"]
    assert cost["plain_f32_cost_over_closure_cost"] == pytest.approx(
        r ** 4 * mlups["f16dev+closure"]["mlups"] / mlups["f32"]["mlups"], rel=1e-2)
