"""Host checks of bench.py's command line: one GPU only, named profiling legs,
and the traffic figure tied to the sweep sources it was measured on."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = run_bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr


def test_unknown_leg_is_refused():
    r = run_bench("--legs", "batched,nonsense")
    assert r.returncode == 2
    assert "nonsense" in r.stderr


def test_traffic_follows_the_profiled_sources(monkeypatch):
    """traffic_from_profiles returns the recorded HBM bytes of a profiled
    schedule while the sweep sources hash as recorded, and None for an
    unprofiled schedule or once the sources differ."""
    sys.path.insert(0, ROOT)
    import bench

    t = bench.traffic_from_profiles(25)
    assert t is not None and 1.0 < t / (288 * 2048 * 2048) < 1.5
    assert bench.traffic_from_profiles(7) is None
    monkeypatch.setattr(bench, "sweep_source_hash", lambda: "0" * 64)
    assert bench.traffic_from_profiles(25) is None


def test_cpu_baseline_reports_cores_and_host():
    """The oracle baseline carries the all-cores figure (threads actually
    used), the one-thread figure and the host's CPU model and core count."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_1805_07251_amd import inputs as I

    cb = bench.cpu_baseline(I.spinodal_small(0, n=32), legs=False, steps_all=2, steps_one=1)
    assert cb["kind"] == "oracle" and cb["unit"] == "MLUPS×C" and cb["value"] > 0
    assert cb["cores"] >= 1 and cb["single_thread"]["cores"] == 1 and cb["single_thread"]["value"] > 0
    assert cb["host"]["nproc"] >= 1 and isinstance(cb["host"]["model"], str)
