"""Parity of the single-graph path under injected delays. The race-testing
build of the library pauses each wave for a varying time before every link CAS
and path-splitting store, which widens the windows in which other waves change
the same entries; the labels must still be the oracle's. The library is chosen
when the package loads, so the cases run in a child process
(tests/stress_delays_run.py) with CCMI_LIBRARY set to that build."""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
STRESS = os.path.join(ROOT, "paper_2507_03695_amd", "libccmi_stress.so")


def test_parity_with_injected_delays():
    assert os.path.exists(STRESS), "libccmi_stress.so is missing: run __graft_entry__.build()"
    env = dict(os.environ, CCMI_LIBRARY=STRESS)
    r = subprocess.run([sys.executable, "-u", os.path.join(HERE, "stress_delays_run.py")],
                       env=env, capture_output=True, text=True, timeout=280)
    print(r.stdout[-3000:])
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
