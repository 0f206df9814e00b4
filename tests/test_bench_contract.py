"""CPU checks of bench.py's contract: one GPU only (--gpus above 1 exits with a message), and
the committed traffic summary matches the rate kernel's sources (so the line's `traffic` is
not null)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_summary_matches_the_kernel_sources():
    import bench
    t = bench.traffic_from_profile()
    assert t is not None, "profiles/traffic_rates32_porous256.md was taken on other sources"
    assert t["bytes"] == t["read_bytes"] + t["write_bytes"] > 0
