"""Host test of the serving loop's device-memory arena (first fit with coalescing), compiled
with g++ from the library's own header and run on the CPU."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_arena_native(tmp_path):
    exe = tmp_path / "arena_test"
    src = os.path.join(HERE, "native", "arena_test.cpp")
    cc = subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-fsanitize=address,undefined",
                         src, "-o", str(exe)], capture_output=True, text=True)
    if cc.returncode != 0:
        pytest.fail(cc.stderr)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stderr
    assert "arena ok" in r.stdout
