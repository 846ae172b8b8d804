"""Host checks of the persisted tuning cache: the C++ reader and writer
(csrc/ga_tune_cache.hpp, the code ga_plan_tune uses) built with g++ under
AddressSanitizer and UndefinedBehaviorSanitizer and run on the CPU (round
trips, malformed files refused and left untouched, merges of keys), and the
written file read back as JSON."""

import json
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_tune_cache_under_host_sanitizers(tmp_path):
    exe = str(tmp_path / "tune_cache_check")
    cmd = ["g++", "-std=c++17", "-Wall", "-Wextra", "-Werror", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "paper_1711_05017_amd", "csrc"),
           os.path.join(ROOT, "tests", "native", "tune_cache_check.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    work = tmp_path / "scratch"
    work.mkdir()
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe, str(work)], capture_output=True, text=True, env=env, timeout=120)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.startswith("OK\n")
    cache = json.loads(res.stdout[3:])
    assert set(cache) == {"gfx950/128/64/1", "gfx950/64/16/1", "gfx950/192/8/1"}
    assert cache["gfx950/128/64/1"] == {"groups": 4, "k": 4, "xcd": 2, "radix": 0, "overlap": 2, "us": 806.125}
    assert json.loads((work / "tune.json").read_text()) == cache
    assert not [p for p in os.listdir(work) if ".tmp." in p]  # no temporary files left
