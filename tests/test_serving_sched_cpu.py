"""The serving loop's scheduler on the CPU, with a fake executor.

serving_sched.h holds the host-side part of hs_server: the first-fit device
arena and the admission / completion bookkeeping. sched_check.cpp drives it
with a fake executor (requests "run" for a number of steps, or finish on a
worker thread as HIP stream callbacks do) and checks that the arena budget is
never exceeded and its free list stays coalesced, that arrival order is kept
under FIFO admission, that a waiting request is passed at most max_bypass
times under bypass admission (and is passed at all), that slots are reused
only after their request finished, that a failed start completes at once and
frees its space, and that requests larger than the arena are refused. The
program is built three times: plain, with AddressSanitizer and
UndefinedBehaviorSanitizer, and with ThreadSanitizer.
"""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "sched_check.cpp")

BUILDS = {
    "plain": ["-O2"],
    # sanitizer runtimes linked statically, so they come first whatever the
    # process environment preloads
    "asan_ubsan": ["-O1", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer",
                   "-fno-sanitize-recover=undefined", "-static-libasan", "-static-libubsan"],
    "tsan": ["-O1", "-g", "-fsanitize=thread", "-static-libtsan"],
}


@pytest.mark.parametrize("build", list(BUILDS))
def test_scheduler_checks(build, tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path / f"sched_{build}")
    cmd = [gxx, "-std=c++17", "-Wall", "-Werror", *BUILDS[build], SRC, "-o", exe, "-pthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0"
    env["TSAN_OPTIONS"] = "halt_on_error=1"
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all scheduler checks passed" in r.stdout
    assert "WARNING: ThreadSanitizer" not in r.stderr
    assert "ERROR: AddressSanitizer" not in r.stderr
