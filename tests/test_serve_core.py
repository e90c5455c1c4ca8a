"""Host logic of the serving loop (admission, FIFO, budget, failures,
continuous batching, drain) with a fake executor, compiled with g++ and run
on the CPU (no GPU). Also built with the host sanitizers."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpp", "test_serve_core.cpp")


@pytest.mark.parametrize("san", [[], ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"],
                                 ["-fsanitize=thread"]], ids=["plain", "asan_ubsan", "tsan"])
def test_serve_core(tmp_path, san):
    exe = tmp_path / "serve_core"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-pthread", *san, "-I", os.path.join(HERE, "..", "include"),
           SRC, "-o", str(exe)]
    subprocess.run(cmd, check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "serve core tests passed" in r.stdout
