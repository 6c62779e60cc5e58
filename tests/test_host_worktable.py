"""Host logic of the library on the CPU: the inter-body work table
(paper_1406_0236_amd/csrc/worktable.h, host C++ only) compiled with g++ and
checked on seeded random bodies by tests/host/worktable_check.cpp."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_work_table_partitions_targets_and_covers_other_bodies(tmp_path):
    exe = tmp_path / "worktable_check"
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-o", str(exe),
                           os.path.join(HERE, "host", "worktable_check.cpp")])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.startswith("ok ")
