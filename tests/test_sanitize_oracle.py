"""The C oracle built with AddressSanitizer and UndefinedBehaviorSanitizer
(gcc) and driven through every entry point on small and ragged grids, both
boundary rules (tests/sanitize/oracle_driver.c): no out-of-bounds access,
leak or undefined arithmetic may be reported.  CPU only; the sanitizers
run in a standalone executable, not inside the Python process."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_is_clean_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    srcs = [os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
            os.path.join(ROOT, "oracle", "rd3d_oracle.c"), os.path.join(ROOT, "oracle", "jacobi_oracle.c")]
    cc = subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                         "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wall", "-Wextra",
                         "-o", exe, *srcs, "-lm"], capture_output=True, text=True)
    assert cc.returncode == 0, cc.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    print(run.stdout, run.stderr)
    assert run.returncode == 0, run.stdout + run.stderr
    assert "oracle driver: ok" in run.stdout
    assert "ERROR: AddressSanitizer" not in run.stderr and "runtime error" not in run.stderr
