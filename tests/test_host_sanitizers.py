"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer: the MPO
builders (csrc/mpo.cpp, plain host C++) are compiled with g++ and the
sanitizers, and a driver calls every builder and charge table over chain
lengths 1-17 and ranges 1-5 with outputs in buffers of exactly the
announced size.  A sanitizer report or a failed invariant fails the test.
(The HIP sources' host code is exercised by the rest of the suite; their
device code cannot be built with sanitizers here.)"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_mpo_builders_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "mpo_driver")
    # the sanitizer runtimes are linked statically, so the executable runs in
    # whatever process environment the test runs in
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-static-libasan", "-static-libubsan",
           os.path.join(ROOT, "tests", "host_sanitizer", "mpo_driver.cpp"),
           os.path.join(ROOT, "paper_1501_05504_amd", "csrc", "mpo.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and r.stdout.strip() == "ok", (r.stdout[-2000:], r.stderr[-4000:])
