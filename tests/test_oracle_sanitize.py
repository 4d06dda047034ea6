"""The oracle built with the host address and undefined-behaviour sanitizers
(g++, CPU only): a driver runs every oracle entry point on small periodic,
superposed and Dirichlet blocks with every face type; the run must be clean
(no sanitizer report, exit status 0) and every result finite."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_sanitizer_build(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    flags = ["-O1", "-g", "-std=c++17", "-fopenmp", "-fno-omit-frame-pointer",
             "-fsanitize=address", "-fsanitize=undefined", "-fno-sanitize-recover=all"]
    cmd = ["g++", *flags, os.path.join(HERE, "sanitize", "oracle_driver.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    # (a library preloaded by the environment may come before the sanitizer
    # runtime in the link order; the order check is switched off, nothing else)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "clean" in r.stdout
    assert "runtime error" not in out and "AddressSanitizer" not in out, out[-4000:]
