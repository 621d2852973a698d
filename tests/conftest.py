import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) and the built HIP library")


def report_path(name):
    """Where GPU tests write their JSON reports: $TRAJ_REPORT_DIR (default
    test_reports/ at the repository root), created on demand."""
    d = os.environ.get("TRAJ_REPORT_DIR", os.path.join(ROOT, "test_reports"))
    os.makedirs(d, exist_ok=True)
    return os.path.join(d, name)
