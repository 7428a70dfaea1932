"""Host test of the uplift server's scheduling policy (serve_sched.h): built
with g++ and run with a stand-in executor; no GPU.  Also built with
ThreadSanitizer (the concurrent-workers case must be free of data races)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2410_14462_amd", "csrc")


def build_and_run(tmp_path, name, flags):
    exe = str(tmp_path / name)
    subprocess.run(["g++", "-std=c++17", "-pthread", *flags, "-I", CSRC,
                    os.path.join(HERE, "serve_sched_test.cpp"), "-o", exe], check=True)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    return r


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_scheduler_policy(tmp_path):
    r = build_and_run(tmp_path, "serve_sched_test", ["-O1"])
    assert r.returncode == 0, r.stderr
    assert r.stdout.startswith("ok")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_scheduler_policy_under_thread_sanitizer(tmp_path):
    r = build_and_run(tmp_path, "serve_sched_tsan", ["-O1", "-g", "-fsanitize=thread"])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "WARNING: ThreadSanitizer" not in r.stderr
    assert r.stdout.startswith("ok")
