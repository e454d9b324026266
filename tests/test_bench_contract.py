"""Host-side checks of the benchmark script's contract (no GPU needed): more than
one GPU is refused with a message and exit status 2, before any device work."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_options_are_documented():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--help"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 0
    for opt in ("--gpus", "--steps", "--warmup", "--workload", "--schedule", "--mapping", "--paper-protocol",
                "--ablations"):
        assert opt in r.stdout


def test_mapping_must_cover_every_chain_length():
    # the default workload is one chain of N = 100: a mapping for N = 55 only is refused
    # before any device work
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--mapping", "55:0x11", "--steps", "1"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "no code for chain length(s) [100]" in r.stderr
    assert r.stdout.strip() == ""
