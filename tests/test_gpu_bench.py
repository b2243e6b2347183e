"""The benchmark's output contract, on the small 32^3 workload: one JSON line
on stdout with the headline metric, the dominant kernel's roofline and the
CPU oracle leg."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_json_line():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "blackoil32",
                        "--steps", "1", "--warmup", "0", "--variants", "none",
                        "--cpu-budget", "3"],
                       capture_output=True, text=True, timeout=600, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    assert len(lines) == 1, r.stdout
    d = json.loads(lines[0])
    assert d["n_gpus"] == 1 and d["steps"] == 1 and d["warmup"] == 0
    assert d["value"] > 0 and d["unit"] == "s" and d["higher_is_better"] is False
    # value: the mean time to solution of the timed steps; ms_per_step: the
    # bracketed timed region divided by the steps (host synchronisation included)
    assert d["ms_per_step"] == pytest.approx(1000 * d["value"], rel=0.05)
    assert d["vs_baseline"] is None and d["data"] == "synthetic" and d["dtype"] == "f64"
    assert d["config"]["workload"].startswith("blackoil32")
    assert d["iters"] > 0 and d["true_relres"] <= 1e-8
    roof = d["roofline"]
    assert roof["bound"] == "hbm" and roof["unit"] == "GB/s" and roof["peak"] == 8000.0
    # frac is printed to four decimals
    assert 0 < roof["achieved"] and roof["frac"] == pytest.approx(roof["achieved"] / roof["peak"],
                                                                  abs=6e-5)
    assert "traffic" in roof
    cpu = d["cpu_baseline"]
    assert cpu["kind"] == "oracle" and cpu["value"] > 0 and cpu["cores"] >= 1
    assert cpu["unit"] == "s" and cpu["sample"]
