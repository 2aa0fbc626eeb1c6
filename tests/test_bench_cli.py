"""Host-side checks of bench.py's command line: requests it cannot serve end
before anything touches a GPU, with a message and a non-zero status."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    env = dict(os.environ, WORLD_SIZE="1")
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120, env=env, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_batched_hardware_queue_count_is_bounded():
    r = _run("--batched", "--hw-queues", "64")
    assert r.returncode != 0
    assert "--hw-queues" in r.stderr and r.stdout == ""


def test_step_counts_are_checked():
    for args in (("--steps", "0"), ("--warmup", "-1")):
        r = _run(*args)
        assert r.returncode != 0
        assert "--steps must be at least 1" in r.stderr and r.stdout == ""
