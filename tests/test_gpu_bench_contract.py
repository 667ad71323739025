"""The benchmark's one-line JSON contract, run end to end on the GPU on the
small ring workload (2,000 observations, FP64): the required keys and their
types, value = observations x steps / timed seconds, the roofline object
(frac = achieved / peak, the recorded traffic while the kernel sources hash to
the profile's value) and the oracle's CPU baseline."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_json_line_on_the_ring_workload():
    cmd = [sys.executable, os.path.join(ROOT, "bench.py"), "--workload", "ring", "--steps", "5", "--warmup", "2",
           "--no-time-to-rmse"]
    print("running", " ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=240, cwd=ROOT)
    assert r.returncode == 0, r.stderr[-2000:]
    lines = [l for l in r.stdout.strip().splitlines() if l.startswith("{")]
    assert len(lines) == 1
    d = json.loads(lines[0])
    for k, t in (("metric", str), ("value", float), ("unit", str), ("n_gpus", int), ("steps", int),
                 ("warmup", int), ("ms_per_step", float), ("higher_is_better", bool), ("scaling", str),
                 ("dtype", str), ("data", str), ("config", dict), ("roofline", dict), ("cpu_baseline", dict)):
        assert isinstance(d[k], t), k
    assert (d["n_gpus"], d["steps"], d["warmup"]) == (1, 5, 2)
    assert d["higher_is_better"] is True and d["vs_baseline"] is None
    assert d["dtype"] == "f64" and d["data"] == "synthetic"
    cfg = d["config"]
    assert cfg["workload"].startswith("ring") and cfg["n_obs"] == 2000
    assert d["value"] > 0 and d["ms_per_step"] > 0
    assert d["value"] == pytest.approx(cfg["n_obs"] / (d["ms_per_step"] * 1e-3), rel=1e-6)
    rf = d["roofline"]
    assert rf["bound"] in ("alu", "hbm", "mfma") and rf["unit"] in ("TFLOP/s", "GB/s")
    assert rf["bound"] == "hbm" and rf["unit"] == "GB/s" and rf["peak"] == 8000.0
    assert rf["bytes_per_obs"] == 408     # FP64: pixel 16, indexes 8, copies 2 x 96, duals 2 x 96
    assert 0 < rf["achieved"]
    assert rf["achieved"] == pytest.approx(rf["bytes_per_obs"] * cfg["n_obs"] / (rf["avg_launch_ms"] * 1e-3) / 1e9,
                                           rel=1e-3)
    assert rf["frac"] == pytest.approx(rf["achieved"] / rf["peak"], abs=1e-4)
    assert rf["alu"]["nonpacked_peak_tflops"] == 78.6
    sys.path.insert(0, ROOT)
    import bench
    recorded, _ = bench.recorded_traffic("ring")
    assert rf["traffic"] == recorded
    cb = d["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["cores"] == 1 and cb["value"] > 0 and cb["unit"] == d["unit"]
    assert "observations" in cb["sample"]
