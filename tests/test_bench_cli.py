"""bench.py's command line on a machine without a GPU: more than one GPU is
refused with a message before anything touches a device."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_world_size_above_one_is_refused():
    env = dict(os.environ, WORLD_SIZE="4")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")], capture_output=True,
                       text=True, timeout=120, env=env)
    assert r.returncode == 2 and "Use --gpus 1" in r.stderr


def test_cpu_baseline_host_record():
    """The CPU baseline names the host it ran on: a CPU model string and the
    number of CPUs the process may use (at least one)."""
    sys.path.insert(0, ROOT)
    import bench
    h = bench.host_cpu()
    assert isinstance(h["model"], str)
    assert isinstance(h["cpus_available"], int) and h["cpus_available"] >= 1
