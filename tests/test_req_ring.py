"""The serving request ring's host bookkeeping (csrc/req_ring.hpp), built
with the host compiler and checked by a randomised driver: pieces stay in
bounds, aligned and disjoint whatever order they come back in, the ring
wraps in order, and a piece returned out of order frees nothing until the
oldest one is back."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2512_18334_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_request_ring_bookkeeping(tmp_path):
    exe = tmp_path / "req_ring_check"
    subprocess.run(["g++", "-std=c++17", "-O1", "-Wall", "-Werror", "-I", CSRC,
                    os.path.join(HERE, "native", "req_ring_check.cpp"), "-o", str(exe)],
                   check=True, capture_output=True, text=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
