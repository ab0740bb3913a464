import os
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
if str(ROOT) not in sys.path:
    sys.path.insert(0, str(ROOT))

# Achieved errors of the GPU results against their references, collected by the
# parity tests (record_error) and printed as one table at the end of the run.
_ERRORS = {}


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (runs through the HIP C-ABI library)")
    config.addinivalue_line("markers", "slow: larger CPU oracle cases")


@pytest.fixture(scope="session")
def orc():
    from oracle import oracle as o

    return o


@pytest.fixture
def record_error(request):
    """record_error(kind, value): keep the largest achieved error per (test
    function, kind) for the summary printed after the run."""

    def rec(kind, value):
        key = (request.node.originalname or request.node.name, kind)
        _ERRORS[key] = max(float(value), _ERRORS.get(key, 0.0))
        print(f"[err] {request.node.nodeid} {kind} = {float(value):.3e}", flush=True)

    return rec


def pytest_terminal_summary(terminalreporter, exitstatus, config):
    if not _ERRORS:
        return
    terminalreporter.write_line("achieved errors against the references (max over parameter cases):")
    for (name, kind), v in sorted(_ERRORS.items()):
        terminalreporter.write_line(f"  {name:48s} {kind:36s} {v:.3e}")
