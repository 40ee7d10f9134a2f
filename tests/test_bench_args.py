"""bench.py's argument guards, which run before anything touches a GPU: more
than one GPU is refused (this projector measures one GPU's share), and fewer
than two timed steps are refused (alternate steps time the forward's and the
adjoint's kernels).  Both exit with status 2 and a message on stderr."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args],
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU only" in r.stderr and r.stdout == ""


def test_fewer_than_two_steps_is_refused():
    r = _run("--steps", "1")
    assert r.returncode == 2
    assert "--steps 2 or more" in r.stderr and r.stdout == ""
