"""Host logic of the benchmark, on the CPU: the one-GPU contract of --gpus,
the cost model's per-observation figures, the workloads' scene builders, and
the rule that a recorded HBM traffic figure is reported only while the kernel
sources still hash to the value it was taken on."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1708_07954_amd import cost  # noqa: E402


@pytest.mark.parametrize("extra", [["--gpus", "2"], ["--gpus", "8", "--steps", "3"]])
def test_more_than_one_gpu_exits_with_a_message(extra):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *extra], capture_output=True, text=True,
                       timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"] and line["n_gpus_requested"] == int(extra[1])


def test_cost_model_figures():
    # per observation and iteration: 5 LM steps of the 12-unknown problem, and
    # of the Euler camera's 9-unknown problem; the bytes the kernels must move
    assert cost.local_flops_per_obs(5) == 5570
    assert cost.local_flops_per_obs(5, "euler") == 3756
    assert cost.local_flops_per_obs(6) - cost.local_flops_per_obs(5) == cost.LM_STEP
    b32, b64 = cost.bytes_per_obs(True), cost.bytes_per_obs(False)
    assert (b32["local"], b32["consensus"], b32["minimal"]) == (304, 36, 304)
    assert b64["minimal"] == 408
    assert b32["total"] == b32["local"] + b32["consensus"]


def test_kernel_source_hash_and_recorded_traffic(monkeypatch):
    h = bench.kernel_source_hash()
    assert len(h) == 12 and int(h, 16) >= 0
    for wl in ("trajectory", "trajectory_blocks", "trajectory_blocks2", "trajectory_euler", "trajectory_shard8",
               "sphere", "sphere_fp64", "ring", "batched"):
        value, _ = bench.recorded_traffic(wl)
        with open(os.path.join(ROOT, "profiles", bench.COUNTER_SUMMARIES[wl])) as fh:
            recorded_hash = [l.split(":")[1].strip() for l in fh if l.startswith("kernel_source_hash:")][0]
        if recorded_hash == h:
            assert value is not None and 1e6 < value < 2e9
        else:
            assert value is None
    assert bench.recorded_traffic("no_such_workload") == (None, None)
    # one summary, a figure per workload
    if bench.recorded_traffic("sphere")[0] is not None:
        assert bench.recorded_traffic("sphere")[0] < bench.recorded_traffic("sphere_fp64")[0]
    # a kernel change voids the recorded figure
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: "000000000000")
    assert bench.recorded_traffic("trajectory")[0] is None


def test_workload_scenes():
    assert set(bench.WORKLOADS) >= {"trajectory", "trajectory_blocks", "trajectory_euler", "trajectory_shard8",
                                    "batched", "sphere"}
    (shard,) = bench.make_scenes("config2_shard8")
    assert shard.n_points == 25000 and shard.n_cams == 1000
    assert shard.meta["n_ranks"] == 8 and shard.meta["rank"] == 0


def test_profile_summaries_name_their_commands():
    """Each committed profile summary gives the rocprofv3 command that made it,
    runs committed files only, and states the kernel source hash it was taken
    on; every summary the benchmark reads traffic from exists."""
    d = os.path.join(ROOT, "profiles")
    names = sorted(f for f in os.listdir(d) if f.endswith(".md"))
    assert names
    for f in names:
        text = open(os.path.join(d, f)).read()
        assert "rocprofv3" in text and "bench.py" in text, f
        assert "_work/" not in text, f
        assert "kernel_source_hash" in text, f
    for wl, f in bench.COUNTER_SUMMARIES.items():
        assert wl in bench.WORKLOADS and f in names, (wl, f)


def test_kernel_source_hash_covers_every_device_source():
    """The hash that keys the recorded traffic covers every HIP file and every
    header such a file includes, directly or through another header."""
    import re
    csrc = os.path.join(ROOT, "paper_1708_07954_amd", "csrc")
    seen, todo = set(), [f for f in os.listdir(csrc) if f.endswith(".hip")]
    while todo:
        f = todo.pop()
        if f in seen:
            continue
        seen.add(f)
        text = open(os.path.join(csrc, f)).read()
        todo += [g for g in re.findall(r'#include "([^"]+)"', text) if os.path.exists(os.path.join(csrc, g))]
    assert seen <= set(bench.KERNEL_SOURCES), sorted(seen - set(bench.KERNEL_SOURCES))
