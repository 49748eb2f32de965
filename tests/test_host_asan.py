"""The library's host-side hull code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU):
hull.cpp and a driver (tests/asan/hull_driver.cpp) built with g++ and run over random octahedral
polytopes; the run must finish cleanly with every constraint valid on the hull's points."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no g++")
def test_hull_under_sanitizers(tmp_path):
    exe = str(tmp_path / "hull_asan")
    src = [os.path.join(ROOT, "tests", "asan", "hull_driver.cpp"),
           os.path.join(ROOT, "paper_2205_00263_amd", "csrc", "hull.cpp")]
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined"] + src + ["-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=300)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert r.stdout.startswith("ok "), r.stdout
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
