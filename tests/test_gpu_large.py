"""Full-size parity of the large intersection join (1M blobs x 200k tubes,
tau = 0, host-resident meshes under a 32 GB device cap) in the configuration
bench.py times: every MBB candidate is decided by the oracle.  The join runs
in a process of its own (``large_parity.py``) so that the set can be built by
forked workers before that process opens the GPU."""
import json
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu
HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.timeout(1100)
def test_large_workload_full_parity():
    p = subprocess.run([sys.executable, "-u", os.path.join(HERE, "large_parity.py")], stdout=subprocess.PIPE,
                       text=True, timeout=1000)
    lines = [ln for ln in p.stdout.splitlines() if ln.startswith("{")]
    assert lines, f"no result line (exit {p.returncode})"
    out = json.loads(lines[-1])
    print(out)
    assert p.returncode == 0 and out["ok"], out
    assert out["candidates_oracle"] > 100 and out["results"] > 10
