"""The search's batch-merge comparator networks (csrc/kbmi_merge_network.h):
the committed header is what its generator writes, and the compiled networks,
applied with the kernel's semantics, return the best KM of list + batch in
descending order for every list length."""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_1901_02492_amd", "csrc")


def test_header_matches_generator():
    with tempfile.TemporaryDirectory() as d:
        out = os.path.join(d, "net.h")
        subprocess.run([sys.executable, os.path.join(CSRC, "gen_merge_network.py"), out],
                       check=True, capture_output=True)
        assert open(out).read() == open(os.path.join(CSRC, "kbmi_merge_network.h")).read()


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_networks_merge_correctly():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "check")
        subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC,
                        os.path.join(os.path.dirname(__file__), "merge_network_check.cpp"),
                        "-o", exe], check=True)
        r = subprocess.run([exe], capture_output=True, text=True)
        assert r.returncode == 0, r.stdout + r.stderr
