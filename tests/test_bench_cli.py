"""Host-only checks of bench.py's command line (no GPU): more than one GPU is
refused with a message, and the help lists the flags the measurements use."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = _bench("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_help_lists_the_measurement_flags():
    r = _bench("--help")
    assert r.returncode == 0
    for flag in ("--steps", "--warmup", "--gpus", "--learned-only", "--cdf97-only", "--lp-points", "--no-cpu-baseline"):
        assert flag in r.stdout, flag
