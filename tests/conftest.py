import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")
    config.addinivalue_line("markers", "slow: long-running CPU test")


def pytest_sessionfinish(session, exitstatus):
    """With GLLMG_PARITY_REPORT=<path>, write the plain relative errors of every FP64 parity
    comparison (and how much of its bar each used) as JSON."""
    path = os.environ.get("GLLMG_PARITY_REPORT")
    if not path:
        return
    mod = sys.modules.get("gpu_helpers")
    rows = list(getattr(mod, "OBSERVED", [])) if mod else []
    import json
    with open(path, "w") as f:
        json.dump(rows, f, indent=0)
