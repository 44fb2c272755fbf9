"""bench.py's command-line contract on the CPU: more than one GPU is refused
with a message (this build is one-GPU), and --help lists the options."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode != 0
    assert "one GPU" in out.stderr


def test_help_lists_the_options():
    out = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"], capture_output=True,
                         text=True, timeout=120)
    assert out.returncode == 0
    for opt in ("--gpus", "--steps", "--warmup", "--workload", "--no-variants", "--paper-sizes",
                "--serve-inflight", "--serve-reserve-cus"):
        assert opt in out.stdout, opt
