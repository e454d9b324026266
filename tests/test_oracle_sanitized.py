"""The oracle's pin tests once more, against an AddressSanitizer and
UndefinedBehaviorSanitizer build of the same C source (CPU only): an
out-of-bounds access, a use after free, a signed overflow, a misaligned or
null access or a shift out of range anywhere on the paths the pins exercise
(energies, trees, Philox, draws, the log, whole runs with logs, series,
exchanges and restarts) ends the run with a sanitizer report.  The
quadrature tests of the N = 2 and N = 3 chains are left out: they run the
same code paths as the pins for 3x10^5 sweeps, which under the sanitizers
would take the CPU suite well past a few minutes."""
import os
import shutil
import subprocess
import sys

import pytest

from oracle import build as ob

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    path = subprocess.run(["gcc", f"-print-file-name={name}"], stdout=subprocess.PIPE, text=True).stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.timeout(900)
def test_oracle_pins_under_asan_and_ubsan(tmp_path):
    if shutil.which("gcc") is None or _runtime("libasan.so") is None:
        pytest.skip("gcc with the AddressSanitizer runtime is not available")
    lib = ob.build(sanitize=True, out=str(tmp_path / "liboracle_asan.so"))
    env = dict(os.environ)
    env["PT_ORACLE_LIB"] = lib
    # The sanitizer runtime must come first in a process that dlopens the
    # sanitized library; the interpreter's own allocations are not checked
    # for leaks.
    env["LD_PRELOAD"] = _runtime("libasan.so")
    env["ASAN_OPTIONS"] = "detect_leaks=0:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["OMP_NUM_THREADS"] = "4"
    cmd = [sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
           "tests/test_oracle_pins.py", "tests/test_pair_enumeration.py"]
    r = subprocess.run(cmd, cwd=ROOT, env=env, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = r.stdout
    print(out[-3000:])
    assert "AddressSanitizer" not in out and "runtime error:" not in out, out[-6000:]
    assert r.returncode == 0, out[-6000:]
    assert " passed" in out
