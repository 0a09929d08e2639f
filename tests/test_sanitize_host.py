"""libdcp's host code built with AddressSanitizer and
UndefinedBehaviorSanitizer (device code unchanged) and driven through every
host-only call (tests/sanitize/host_driver.cpp): no out-of-bounds access,
leak in the library's own code or undefined arithmetic may be reported.
CPU only.  About two minutes of compilation: runs with DCP_SANITIZE_HOST=1."""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2107_00555_amd", "csrc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer"]


@pytest.mark.skipif(os.environ.get("DCP_SANITIZE_HOST") != "1",
                    reason="about two minutes of compilation; set DCP_SANITIZE_HOST=1")
def test_host_code_is_clean_under_asan_and_ubsan(tmp_path):
    from paper_2107_00555_amd import build
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off", f"--offload-arch={build.ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             f"-I{os.path.join(ROOT, 'include')}", f"-I{CSRC}"] + SAN

    def compile_one(src):
        obj = str(tmp_path / (os.path.splitext(os.path.basename(src))[0] + ".o"))
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        r = subprocess.run([hipcc] + lang + flags + ["-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        return obj

    srcs = [os.path.join(CSRC, s) for s in build.SOURCES] + [os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp")]
    with ThreadPoolExecutor(8) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(tmp_path / "host_driver")
    r = subprocess.run([hipcc, f"--offload-arch={build.ARCH}"] + SAN + ["-o", exe] + objs + ["-lhiprtc"],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
    supp = os.path.join(ROOT, "tests", "sanitize", "lsan.supp")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1",
               LSAN_OPTIONS=f"suppressions={supp}:print_suppressions=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=900)
    print(run.stdout, run.stderr[-4000:])
    assert run.returncode == 0, run.stdout + run.stderr[-4000:]
    assert "host driver:" in run.stdout
    assert "ERROR: AddressSanitizer" not in run.stderr and "runtime error" not in run.stderr
    assert "ERROR: LeakSanitizer" not in run.stderr
