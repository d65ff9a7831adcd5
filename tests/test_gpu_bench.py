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
