"""Host code under the sanitizers (CPU only): the oracle's C entry points,
the schedule tables (plan.cpp) and the server's queue/admission core
(serve_core.cpp, driven by a host-only backend from several threads), each
built with g++/gcc and AddressSanitizer + UndefinedBehaviorSanitizer, and
the server core again with ThreadSanitizer.  The drivers under
tests/sanitize/ check plain properties of what they run and exit 0 only
when every check holds; any sanitizer report fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2509_02840_amd", "csrc")
ASAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
TSAN = ["-O1", "-g", "-fsanitize=thread"]
HIP_HOST = ["-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include"]

CASES = {
    "oracle_asan": (["gcc", "-std=c11", *ASAN, os.path.join(ROOT, "oracle", "bgu_oracle.c"),
                     os.path.join(SAN, "oracle_driver.c"), "-lm"], "oracle: all checks passed"),
    "plan_asan": (["g++", "-std=c++17", *ASAN, *HIP_HOST, os.path.join(CSRC, "plan.cpp"),
                   os.path.join(SAN, "plan_driver.cpp")], "plan: all checks passed"),
    "serve_asan": (["g++", "-std=c++17", *ASAN, "-pthread", os.path.join(CSRC, "serve_core.cpp"),
                    os.path.join(SAN, "serve_driver.cpp")], "serve core: all checks passed"),
    "serve_tsan": (["g++", "-std=c++17", *TSAN, "-pthread", os.path.join(CSRC, "serve_core.cpp"),
                    os.path.join(SAN, "serve_driver.cpp")], "serve core: all checks passed"),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_sanitized_driver(case, tmp_path):
    cmd, ok = CASES[case]
    if shutil.which(cmd[0]) is None:
        pytest.skip(f"{cmd[0]} not available")
    exe = str(tmp_path / case)
    b = subprocess.run([*cmd, "-o", exe], capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1",
               TSAN_OPTIONS="halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report[-4000:]
    assert ok in r.stdout
    for marker in ("ERROR: AddressSanitizer", "runtime error:", "WARNING: ThreadSanitizer", "ERROR: LeakSanitizer"):
        assert marker not in report, report[-4000:]
