"""The learned contact-time bracket never changes the contact (host build of
the library's narrow-phase header).

The search of Eq. 3.1 with a predicted bracket [lo, hi] and start point must
return the earliest valid root that the plain subdivision search returns,
for good, skewed, random, early, late and boundary predictions, with d > 0
and d = 0.  tests/host_bracket.cpp runs 2 x 20 000 random vertex-triangle
and edge-edge quads, 7 predictions each, compiled for the host with hipcc
(no GPU code runs).
"""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1812_04719_amd", "csrc")


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_bracketed_search_equals_plain_host_build():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "bracket")
        subprocess.check_call(["hipcc", "-x", "hip", "--offload-host-only", "-O2", "-std=c++17",
                               "-ffp-contract=off", "-I" + CSRC, os.path.join(HERE, "host_bracket.cpp"),
                               "-o", exe])
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
        print(r.stdout)
        assert r.returncode == 0, r.stdout + r.stderr
        assert r.stdout.strip().endswith("OK")
        used = int(r.stdout.split("bracket used ")[1].split()[0])
        assert used > 10000  # the bracketed path is exercised, not only the plain one
