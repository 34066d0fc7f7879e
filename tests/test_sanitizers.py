"""Host sanitizer run (AddressSanitizer and UndefinedBehaviorSanitizer) of the C code the tests
rely on: the oracle (oracle/scqr_oracle.c) and the compensated accuracy metrics
(accuracy/scqr_accuracy.c), every entry point on small inputs through tests/sanitize_driver.c.
Any out-of-bounds access, use after free, leak, signed overflow or misaligned access fails the
test.  CPU only: nothing here touches a GPU."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_and_accuracy_under_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_driver")
    cmd = ["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-fopenmp",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "sanitize_driver.c"), os.path.join(ROOT, "accuracy", "scqr_accuracy.c"),
           "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, OMP_NUM_THREADS="2",
               ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert "runtime error" not in res.stderr and "ERROR: AddressSanitizer" not in res.stderr, res.stderr
    assert "ok" in res.stdout
