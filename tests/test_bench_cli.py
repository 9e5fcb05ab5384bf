"""bench.py's command line on the host: one JSON line, and a clear refusal
for more than one GPU or for a machine without one (no GPU needed)."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run_bench(*args, env=None):
    e = dict(os.environ)
    if env:
        e.update(env)
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                       cwd=ROOT, env=e, timeout=300)
    lines = [ln for ln in p.stdout.splitlines() if ln.strip()]
    return p.returncode, lines


def test_more_than_one_gpu_is_refused():
    rc, lines = run_bench("--gpus", "2")
    assert rc == 2
    assert len(lines) == 1
    assert "one GPU" in json.loads(lines[0])["error"]


def test_world_size_above_one_is_refused():
    rc, lines = run_bench(env={"WORLD_SIZE": "2"})
    assert rc == 2
    assert "one GPU" in json.loads(lines[0])["error"]


def test_no_gpu_is_reported():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    rc, lines = run_bench("--steps", "1", "--warmup", "0")
    assert rc == 1
    assert len(lines) == 1
    assert json.loads(lines[0]) == {"error": "no GPU visible"}
