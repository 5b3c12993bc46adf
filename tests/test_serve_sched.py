"""Host bookkeeping of the serving loop, on the CPU: the scheduler header is
compiled with g++ (no HIP) into a small checker that drives it with
simulated device completions."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("sched") / "sched_check")
    cmd = ["g++", "-O1", "-g", "-std=c++17", "-Wall", "-Werror", "-fsanitize=address,undefined",
           "-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_1905_13415_amd", "csrc"),
           os.path.join(HERE, "sched_check.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def test_scheduler_checks(checker):
    r = subprocess.run([checker], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = r.stdout.split("\n")
    for name in ("arena_model", "admission_fifo", "slots_bound", "budget_and_args", "reparse", "soak"):
        assert any(l.startswith("ok " + name) for l in lines), r.stdout
