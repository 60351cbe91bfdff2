import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")
    config.addinivalue_line("markers", "fullsize: GPU test at the full benchmark lattice sizes")


def pytest_sessionfinish(session, exitstatus):
    """Write the parity errors the GPU tests measured (with their bounds) to
    gpurun_out/parity_errors.json when that folder exists."""
    try:
        import gpu_util
    except Exception:
        return
    out = os.path.join(ROOT, "gpurun_out")
    if gpu_util.MEASURED and os.path.isdir(out):
        import json
        with open(os.path.join(out, "parity_errors.json"), "w") as f:
            json.dump([{"test": t, "norm": n, "site": s, "bound": b} for t, n, s, b in gpu_util.MEASURED], f, indent=0)
