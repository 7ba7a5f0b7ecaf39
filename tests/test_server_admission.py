"""Host-only checks of the evaluation server's staging arena and admission
policy (`csrc/server_admission.hpp`): aligned, disjoint placements inside
the arena and full coalescing on release; arrival order while requests
fit; small requests admitted past a blocked head of the line at the
arena's top end, at most kMaxBypass per head, and the head first once
space frees; the optional cap on large requests active at once;
randomized traffic (with and without the cap) that drains completely.  Compiled with the
host C++ compiler (no GPU, no HIP runtime)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2606_24154_amd", "csrc")


def test_admission_policy(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path / "admission_check")
    subprocess.run([cxx, "-std=c++17", "-O1", "-Wall", "-Werror", "-I", CSRC,
                    os.path.join(HERE, "host", "admission_check.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "checks passed" in r.stdout, r.stdout + r.stderr
