"""The polynomial coefficient header of the element kernels is the current
output of its generator (40-digit Chebyshev interpolation); CPU only."""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2606_24154_amd", "csrc")


def test_poly_coeffs_header_is_generated():
    out = subprocess.run([sys.executable, os.path.join(CSRC, "gen_poly.py")], capture_output=True, text=True,
                         check=True, cwd=CSRC, timeout=300).stdout
    with open(os.path.join(CSRC, "poly_coeffs.hpp")) as f:
        assert f.read() == out
