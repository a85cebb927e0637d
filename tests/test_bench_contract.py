"""Host checks of bench.py's contract that need no GPU: more than one GPU is
refused with a message (the library has no multi-GPU path), and the sweep
kernel named in the roofline follows GSIS_SWEEP_V4."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_roofline_kernel_name(monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    monkeypatch.delenv("GSIS_SWEEP_V4", raising=False)
    assert bench.sweep_kernel_name() == "k_sweep_v4"
    monkeypatch.setenv("GSIS_SWEEP_V4", "0")
    assert bench.sweep_kernel_name() == "k_sweep_fast"
