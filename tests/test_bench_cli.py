"""bench.py's command-line contract on the host: more than one GPU is refused
with a message and exit status 2 before anything touches a device, and every
mode is listed."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*argv):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], cwd=ROOT,
                          capture_output=True, text=True, timeout=120)


def test_more_than_one_gpu_is_refused():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_modes_are_listed():
    r = _run("--help")
    assert r.returncode == 0
    for mode in ("build", "dsweep", "screen", "batched", "wsweep", "quality", "density", "recheck"):
        assert mode in r.stdout
