"""bench.py's contract on the host: it runs on one GPU only and says so."""
from __future__ import annotations

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(args, env=None):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, env=env)


def test_more_than_one_gpu_exits_with_a_message():
    r = _run(["--gpus", "2"])
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
    assert r.stdout == ""


def test_launched_with_several_ranks_exits_with_a_message():
    env = dict(os.environ, WORLD_SIZE="8")
    r = _run(["--gpus", "1"], env=env)
    assert r.returncode == 2
    assert "one GPU only" in r.stderr
