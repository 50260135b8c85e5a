"""Host-side checks of bench.py: the one-GPU contract and the bounded CPU
sample of the oracle baseline (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_cpu_baseline_sample_is_bounded():
    import bench

    r = bench.cpu_baseline(32, 2, target_s=0.2, max_steps=6)
    assert r["kind"] == "oracle" and r["unit"] == "site-steps/s"
    assert r["cores"] >= 1 and r["value"] > 0
    steps = int(r["sample"].split()[0])
    assert 1 <= steps <= 6
    assert "32^3" in r["sample"]


def test_traffic_is_reported_only_for_the_profiled_workload():
    import json

    import bench

    with open(bench.TRAFFIC_FILE) as f:
        t = json.load(f)
    k = t["kernels"]["step_x_fp64"]
    if t["kernel_hash"] == bench.kernel_hash():
        assert bench.traffic_for("step_x_fp64", k["algorithmic_bytes_per_launch"]) == \
            k["hbm_bytes_per_launch"]
    # another grid (1024^3: 8x the bytes) or another kernel: no figure
    assert bench.traffic_for("step_x_fp64", 8 * k["algorithmic_bytes_per_launch"]) is None
    assert bench.traffic_for("no_such_kernel", k["algorithmic_bytes_per_launch"]) is None
