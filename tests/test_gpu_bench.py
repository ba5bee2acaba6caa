"""The benchmark's JSON line on the smallest workload (8^3x8, FP64): the keys of its contract,
a positive rate, the roofline record, the oracle baseline, and the GPU result against the
oracle."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.skip("no GPU")
    return t


def test_bench_line_small_workload(torch):
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "0", "--steps", "2", "--warmup", "1",
           "--no-plain", "--no-w12", "--no-extra"]
    res = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stderr[-3000:]
    d = json.loads(res.stdout.strip().splitlines()[-1])
    for key in ("metric", "value", "unit", "n_gpus", "steps", "warmup", "ms_per_step", "higher_is_better",
                "scaling", "vs_baseline", "dtype", "data", "config", "roofline", "cpu_baseline", "accuracy"):
        assert key in d, key
    assert d["n_gpus"] == 1 and d["steps"] == 2 and d["warmup"] == 1
    assert d["value"] > 0 and d["ms_per_step"] > 0 and d["higher_is_better"] is True
    assert d["unit"] == "RHS-site-updates/s" and d["dtype"] == "f64" and d["data"] == "synthetic"
    assert d["config"]["workload"].startswith("8^3x8")
    r = d["roofline"]
    for key in ("bound", "achieved", "peak", "unit", "frac", "traffic"):
        assert key in r, key
    assert r["bound"] == "hbm" and r["unit"] == "GB/s" and r["peak"] == 8000.0
    assert 0 < r["frac"] == pytest.approx(r["achieved"] / r["peak"], abs=1e-4)   # frac has 4 decimals
    c = d["cpu_baseline"]
    assert c["kind"] == "oracle" and c["value"] > 0 and c["cores"] >= 1 and c["sample"]
    assert c["single_thread"]["cores"] == 1 and c["single_thread"]["value"] > 0
    assert d["accuracy"]["max_rel"] < 1e-12 and d["finite"] is True
