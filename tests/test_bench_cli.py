"""The bench script's command line on the CPU: more than one GPU is refused
with a message before anything touches a device, and the host description
that accompanies the CPU baseline is well formed."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_world_size_above_one_is_refused():
    env = dict(os.environ, WORLD_SIZE="4")
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py")],
                       capture_output=True, text=True, timeout=120, cwd=ROOT, env=env)
    assert p.returncode == 2
    assert "one GPU" in p.stderr


def test_host_description():
    sys.path.insert(0, ROOT)
    import bench
    h = bench._host_cpu()
    assert set(h) == {"model", "cores_available"}
    assert isinstance(h["model"], str) and h["model"]
    assert h["cores_available"] >= 1
