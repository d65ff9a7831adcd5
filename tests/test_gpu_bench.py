"""The benchmark's JSON line keeps its contract (a short run on the small
packing, through the same code path as the headline)."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.parametrize("sweep", ["c8", "c16", "full", "inplace_c16"])
def test_bench_json_contract(sweep):
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "small_packing",
           "--sweep", sweep, "--layout", "aligned", "--steps", "2", "--warmup", "1",
           "--sweeps", "20", "--cpu-seconds", "0.5"]
    print("CASE bench", sweep, flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-2000:]
    d = json.loads(res.stdout.strip().splitlines()[-1])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step",
                "higher_is_better", "scaling", "vs_baseline", "dtype", "data", "config",
                "roofline", "cpu_baseline"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["value"] > 0 and d["unit"] == "MFLUPS" and d["dtype"] == "f64"
    assert d["config"]["sweep"] == sweep and d["config"]["n_fluid"] == 17263
    r = d["roofline"]
    assert r["bound"] == "hbm" and r["peak"] == 8000.0 and r["unit"] == "GB/s"
    assert r["frac"] == pytest.approx(r["achieved"] / r["peak"], abs=1e-4)
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["value"] > 0 and c["cores"] >= 1


def test_bench_sweep_auto_picks_a_kind():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "small_packing",
           "--storage", "f16s", "--sweep", "auto", "--steps", "1", "--warmup", "0",
           "--sweeps", "20", "--cpu-seconds", "0"]
    print("CASE bench auto", flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-2000:]
    d = json.loads(res.stdout.strip().splitlines()[-1])
    from paper_1111_1129_amd.tune import SWEEPS
    assert d["config"]["sweep"] in SWEEPS
    assert "sweep kinds (MFLUPS)" in res.stderr
    assert d["cpu_baseline"] is None


def test_bench_precision_and_crop_baseline():
    """The headline path of the precision workload (edges / 8): the line
    carries every storage form's speed-up and velocity error vs FP64, the
    oracle's rate on the central crop, and every form's error against the
    oracle on that crop."""
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "large_packing",
           "--scale", "8", "--layout", "aligned", "--steps", "1", "--warmup", "1",
           "--sweeps", "40"]
    print("CASE bench precision", flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-2000:]
    d = json.loads(res.stdout.strip().splitlines()[-1])
    assert d["dtype"] == "f64" and d["config"]["workload"].startswith("large_packing")
    p = d["precision"]
    for st in ("f64s", "f32", "f32s", "f16s", "f16s12"):
        for key in ("mflups", "speedup_vs_f64", "u_rel_l2", "u_rel_max", "sweep"):
            assert key in p[st], (st, key)
        assert p[st]["mflups"] > 0 and 0 <= p[st]["u_rel_l2"] < 1
    assert p["f64s"]["u_rel_l2"] < 1e-9          # same arithmetic type, other rounding
    assert p["f32s"]["u_rel_l2"] < p["f32"]["u_rel_l2"]  # the shift keeps FP32 accurate
    crop = p["vs_oracle_on_crop"]
    assert set(crop) == {"f64", "f64s", "f32", "f32s", "f16s", "f16s12"}
    assert crop["f16s12"]["u_rel_l2"] < crop["f16s"]["u_rel_l2"]  # no subnormal deviations
    assert crop["f64"]["u_rel_l2"] < 1e-10 and crop["f64s"]["u_rel_l2"] < 1e-10
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and "crop" in c["sample"] and c["value"] > 0
