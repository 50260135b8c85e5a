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
    assert r["cores"] >= 1 and r["value"] > 0 and r["cpu_model"]
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


class _Clock:
    t = 0.0


class _Event:
    def __init__(self, enable_timing=True):
        self.t = None

    def record(self, stream=None):
        self.t = _Clock.t

    def elapsed_time(self, other):
        return other.t - self.t


class _FakeTorch:
    class cuda:
        Event = _Event

        @staticmethod
        def current_stream():
            return None

        @staticmethod
        def synchronize():
            pass


class _FakeCtx:
    """A context whose steps take 2 ms and whose spectra evaluation 50 ms of
    simulated device time."""

    def __init__(self):
        self.steps, self.evals = 0, 0

    def evolve(self, dt, n):
        self.steps += n
        _Clock.t += 2.0 * n

    def spectra(self, with_obs=False):
        self.evals += 1
        _Clock.t += 50.0

    def timing(self, on=None):
        return None if on is not None else {}


def test_spectra_cost_is_charged_at_its_cadence():
    """20 timed steps of a 100-step cadence owe 0.2 of an evaluation; 250
    steps reach two evaluations and owe half of a third."""
    import bench

    for steps, reached, owed in ((20, 0, 0.2), (250, 2, 0.5), (200, 2, 0.0)):
        ctx = _FakeCtx()
        r = bench.run_workload(ctx, _FakeTorch, steps, 5, 1e-3, 100, True)
        assert r["nspec"] == reached and abs(r["owed"] - owed) < 1e-12
        assert abs(r["ms"] - (2.0 * steps + 50.0 * steps / 100)) < 1e-9
        assert ctx.steps == steps + 5
    r = bench.run_workload(_FakeCtx(), _FakeTorch, 20, 5, 1e-3, 100, False)
    assert r["ms"] == 40.0 and r["owed"] == 0.0
