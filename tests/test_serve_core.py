"""Host logic of the serving loop, built with g++ and run on the CPU: the
arena allocator behind HBM-budget admission (first fit, merging, capacity),
the batch former (same-scene gathering in arrival order, point, request and
budget limits, no overtaking of the oldest request) and the latency
percentile."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))


def test_serve_core(tmp_path):
    exe = tmp_path / "serve_core_check"
    src = os.path.join(HERE, "cpp", "serve_core_check.cpp")
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-o", str(exe), src], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=60)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "serve_core ok" in r.stdout
