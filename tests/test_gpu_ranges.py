"""The range-check build on the GPU: every lazy-range and accumulator bound
the exact arithmetic relies on holds on every path, at the arithmetic's
edges.

tests/range_check_run.py runs in a process of its own with
KS_LIBRARY=libks_check.so (the same kernels with each bound tested where it
is used, violations counted on the device).  It must show the counters live
(the strict REDC bound, which ordinary inputs violate, is counted), return
results equal to the oracle's on every path, and count no violation.
"""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_no_range_violation_on_any_path():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    lib = os.path.join(ROOT, "paper_2311_01598_amd", "libks_check.so")
    assert os.path.exists(lib), "libks_check.so is not built (the package build makes it)"
    env = dict(os.environ, KS_LIBRARY="libks_check.so")
    print("[ranges] running tests/range_check_run.py on libks_check.so", flush=True)
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "tests", "range_check_run.py")], env=env,
                       capture_output=True, text=True, timeout=600)
    sys.stderr.write(r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-2000:]
    res = json.loads(r.stdout.strip().splitlines()[-1])
    print(res, flush=True)
    assert res["library"] == "libks_check.so"
    assert res["strict_count"] > 0 and res["strict_code"] == 6, res  # KS_RC_REDC_OUT
    assert res["checked"] >= 60 and not res["mismatches"], res
    assert res["violations"] == 0, res
