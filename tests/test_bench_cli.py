"""Host-only checks of the benchmark's command line (no GPU is touched)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""



def test_link_summary():
    # runs out and back at the link's published rate bound a spilling step
    sys.path.insert(0, ROOT)
    import bench
    h = bench.link_summary(1_000_000_000, 40.0, 80.0)
    assert h["bytes_per_step"] == 2_000_000_000
    assert h["GBps"] == 50.0
    assert h["frac"] == round(50.0 / bench.LINK_PEAK_GBS, 3)
    assert h["floor_ms_per_step"] == round(2e9 / (bench.LINK_PEAK_GBS * 1e9) * 1e3, 2)
    assert h["step_frac_of_floor"] == round(h["floor_ms_per_step"] / 80.0, 3)
    assert bench.link_summary(10, 0.0, 1.0)["GBps"] is None
