"""The benchmark's host-only modes: the CPU oracle baseline (--cpu-only) on a
small grid of the headline family, and the refusal of several GPUs."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], cwd=ROOT,
                          capture_output=True, text=True, timeout=300, env=env)


def test_cpu_only_line():
    env = dict(os.environ, OMP_NUM_THREADS="2")
    p = run_bench("--cpu-only", "--side", "24", env=env)
    assert p.returncode == 0, p.stderr
    line = json.loads(p.stdout.strip().splitlines()[-1])
    cb = line["cpu_baseline"]
    assert cb["kind"] == "oracle" and cb["unit"] == "s" and cb["value"] > 0
    assert cb["cores"] == 2
    assert "benchmark's own workload" in cb["sample"]


def test_several_gpus_refused():
    p = run_bench("--gpus", "2")
    assert p.returncode == 2
    assert "one GPU" in json.loads(p.stdout.strip().splitlines()[-1])["error"]
