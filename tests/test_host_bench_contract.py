"""The benchmark's command-line contract on the host: it refuses more than one GPU with exit code 2
and a message, and its CPU-baseline leg (the FP64 oracle in a child process) prints one JSON object
with the rate, its unit and the sample it timed."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
BENCH = os.path.join(ROOT, "bench.py")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, BENCH, "--gpus", "2"], capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""  # no bench line


@pytest.mark.parametrize("leg,unit", [("kerr_n20", "solves/s"), ("ising_l8_window", "RHS evals/s")])
def test_cpu_baseline_leg_prints_one_json_object(leg, unit):
    env = dict(os.environ, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, BENCH, "--cpu-leg", leg, "--cpu-budget", "0.2"], capture_output=True,
                       text=True, timeout=300, env=env, check=True)
    out = json.loads(r.stdout.strip().splitlines()[-1])
    assert out["unit"] == unit
    assert out["value"] > 0 and out["seconds"] > 0
    assert isinstance(out["sample"], str) and out["sample"]
