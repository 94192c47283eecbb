"""The benchmark's command line on a host without a GPU: requests it cannot
serve end with a message and a nonzero status before any device work."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_step_counts_are_validated():
    for args in (("--steps", "0"), ("--warmup", "-1")):
        r = _run(*args)
        assert r.returncode == 2 and "--steps must be >= 1" in r.stderr
