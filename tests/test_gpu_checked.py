"""The bounds-checked build of the library (MF_CHECKED) over every instrumented kernel family:
no kernel index may leave its bound.  In that build each instrumented index (LDS slots and rows of
the FFT stages and the spectral, union-of-bases and IUWT kernels; global plane offsets of the IUWT
and union-of-bases kernels; table and visibility indices of the visibility kernels) is compared with its bound on the device; a miss is counted and
replaced by an index in bounds, so the kernels always complete.  The workloads run in one child
process (tests/checked_scenarios.py) that loads paper_1602_08847_amd/libmuffin_checked.so."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CHECKED = os.path.join(ROOT, "paper_1602_08847_amd", "libmuffin_checked.so")


@pytest.mark.timeout(600)
def test_no_kernel_index_leaves_its_bound(lib):
    assert os.path.exists(CHECKED), "build the checked library first (__graft_entry__.build())"
    env = dict(os.environ, MUFFIN_LIBRARY=CHECKED)
    print("[checked] running tests/checked_scenarios.py against", CHECKED, flush=True)
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "tests", "checked_scenarios.py")],
                       capture_output=True, text=True, timeout=540, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    res = json.loads(r.stdout.strip().splitlines()[-1])
    assert res["cases"] >= 39
    assert res["oob"] == 0, res
