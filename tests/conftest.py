import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line(
        "markers", "gpu: needs an MI355X (gfx950) GPU and the built HIP library")


@pytest.fixture(scope="session")
def repo_root():
    return ROOT

# Import torch at collection time so that its first (slow) import on a fresh
# machine does not count against a test's time limit.
try:  # noqa: E402
    import torch  # noqa: F401
except Exception:  # pragma: no cover
    pass
