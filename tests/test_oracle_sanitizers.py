"""The C oracle (test infrastructure) under AddressSanitizer and
UndefinedBehaviorSanitizer: a host driver runs every entry point on small
synthetic inputs (ragged tiles, a camera inside the cloud, row subsets, an
empty scene); any out-of-bounds access, leak or undefined operation fails."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_asan")
    subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fopenmp",
                    os.path.join(ROOT, "oracle", "lv_oracle.c"), os.path.join(HERE, "oracle_sanitize_main.c"),
                    "-o", exe, "-lm"], check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "runtime error" not in r.stderr
    assert r.stdout.startswith("ok")
    print(r.stdout.strip())


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_scheduler_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "sched_asan")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-pthread", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "paper_2410_14462_amd", "csrc"),
                    os.path.join(HERE, "serve_sched_test.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300,
                       env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
    assert r.returncode == 0, r.stderr[-4000:]
    assert r.stdout.startswith("ok")
