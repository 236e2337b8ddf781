"""The CPU oracle and the product's host-side parser / planner built with
AddressSanitizer and UndefinedBehaviorSanitizer (g++, host code only) and
run over small programs of every kind: no report, exit status 0.  The two
are separate programs (the oracle shares no code with the product)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
FLAGS = ["g++", "-std=c++17", "-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
         "-fno-sanitize-recover=all", "-ffp-contract=off"]

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")


def build_and_run(tmp_path, name, sources):
    exe = str(tmp_path / name)
    r = subprocess.run(FLAGS + ["-o", exe] + sources, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("LD_PRELOAD", None)  # the sanitizer runtime must come first
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-6000:])
    assert "runtime error" not in r.stderr and "Sanitizer" not in r.stderr, r.stderr[-6000:]
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    out = build_and_run(tmp_path, "oracle_asan", [os.path.join(HERE, "oracle_driver.cpp"),
                                                  os.path.join(ROOT, "oracle", "naive.cpp"),
                                                  os.path.join(ROOT, "oracle", "special.cpp")])
    assert "oracle driver ok" in out


def test_planner_under_sanitizers(tmp_path):
    out = build_and_run(tmp_path, "planner_asan", [os.path.join(HERE, "planner_driver.cpp"),
                                                   os.path.join(ROOT, "paper_2503_21937_amd", "csrc", "program.cpp")])
    assert "planner driver ok" in out
