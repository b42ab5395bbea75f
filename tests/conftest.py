import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs the HIP path through the C ABI)")
    config.addinivalue_line("markers", "slow: long CPU-oracle runs (excluded from the default CPU suite)")


def pytest_collection_modifyitems(config, items):
    if os.environ.get("PPCWENO_RUN_SLOW"):
        return
    skip = pytest.mark.skip(reason="slow oracle run; set PPCWENO_RUN_SLOW=1")
    for it in items:
        if "slow" in it.keywords:
            it.add_marker(skip)


def pytest_terminal_summary(terminalreporter):
    """List every GPU parity case that used the widened stage bar (the
    oracle's own sensitivity where the limiter holds states on e = eps)."""
    mod = sys.modules.get("test_gpu_parity") or sys.modules.get("tests.test_gpu_parity")
    cases = getattr(mod, "WIDENED", None) if mod else None
    if cases:
        terminalreporter.write_line("widened stage bars (case, bar, limited cells):")
        for c in cases:
            terminalreporter.write_line(f"  {c[0]}: {c[1]:.2e}, {c[2]}")
