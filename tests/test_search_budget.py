"""Root-search budget (host build of the library's narrow-phase header).

The subdivision search of Eq. 3.1 has a budget of intervals per candidate.
A search that runs out of it must be counted as exhausted (the library then
reports STIV_E_NUMERIC), never silently taken for "no contact".  This test
compiles tests/host_search_budget.cpp for the host with hipcc (no GPU code
runs) and checks both a polynomial that exhausts the budget and an ordinary
root.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_1812_04719_amd", "csrc")


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="hipcc not available")
def test_search_budget_host_build():
    with tempfile.TemporaryDirectory() as tmp:
        exe = os.path.join(tmp, "search_budget")
        subprocess.check_call(["hipcc", "-x", "hip", "--offload-host-only", "-O2", "-std=c++17",
                               "-ffp-contract=off", "-I" + CSRC, os.path.join(HERE, "host_search_budget.cpp"),
                               "-o", exe])
        r = subprocess.run([exe], capture_output=True, text=True)
        print(r.stdout)
        assert r.returncode == 0, r.stdout + r.stderr
        assert "fivefold: hit=0 visits=4097 deg=0 exh=1" in r.stdout
